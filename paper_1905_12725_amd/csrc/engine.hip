// Host engine and C ABI of the DBFFT hot path.
//
// One context = one periodic cell: grid, material, FFT plans and twiddles,
// device workspaces, and the current solution.  Every entry point enqueues
// on the context's stream and synchronizes before returning.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstddef>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/dbfft.h"
#include "dbfft_internal.h"
#include "batch.h"
#include "fft_mixed.h"

namespace dbfft {

static thread_local std::string g_err;
constexpr int kMaxSolveStreams = 8;  // helper contexts of dbfft_solve_many
static const bool g_verbose = [] {
  const char* v = std::getenv("DBFFT_VERBOSE");
  return v != nullptr && v[0] != '0';
}();

struct Err {
  int code;
};

#define DB_THROW(code, msg)    \
  do {                         \
    g_err = (msg);             \
    throw Err{(int)(code)};    \
  } while (0)

#define HIPCK(call)                                                                           \
  do {                                                                                        \
    hipError_t e_ = (call);                                                                   \
    if (e_ != hipSuccess) {                                                                   \
      g_err = std::string("HIP error ") + hipGetErrorString(e_) + " at " #call;              \
      throw Err{(int)DBFFT_EHIP};                                                             \
    }                                                                                         \
  } while (0)

static const int kPair[6][2] = {{0, 0}, {1, 1}, {2, 2}, {1, 2}, {0, 2}, {0, 1}};

// ------------------------------------------------------------------ helpers
static bool make_plan(int n, FftPlan& p) {
  std::memset(&p, 0, sizeof(p));
  p.n = n;
  int m = n, ns = 1;
  const int radices[6] = {8, 4, 2, 3, 5, 7};
  for (int r : radices) {
    while (m % r == 0) {
      if (p.nstages >= kMaxStages) return false;
      p.radix[p.nstages] = r;
      p.ns[p.nstages] = ns;
      ns *= r;
      m /= r;
      p.nstages++;
    }
  }
  return m == 1;
}

// inverse of a small dense matrix (row-major, n <= 9), Gauss-Jordan with pivoting
static bool small_inverse(const std::vector<double>& A, int n, std::vector<double>& X) {
  std::vector<double> M(A);
  X.assign(n * n, 0.0);
  for (int i = 0; i < n; ++i) X[i * n + i] = 1.0;
  for (int k = 0; k < n; ++k) {
    int piv = k;
    for (int i = k + 1; i < n; ++i)
      if (std::fabs(M[i * n + k]) > std::fabs(M[piv * n + k])) piv = i;
    if (!(std::fabs(M[piv * n + k]) > 0.0)) return false;
    if (piv != k)
      for (int j = 0; j < n; ++j) {
        std::swap(M[k * n + j], M[piv * n + j]);
        std::swap(X[k * n + j], X[piv * n + j]);
      }
    const double inv = 1.0 / M[k * n + k];
    for (int j = 0; j < n; ++j) {
      M[k * n + j] *= inv;
      X[k * n + j] *= inv;
    }
    for (int i = 0; i < n; ++i) {
      if (i == k) continue;
      const double f = M[i * n + k];
      if (f == 0.0) continue;
      for (int j = 0; j < n; ++j) {
        M[i * n + j] -= f * M[k * n + j];
        X[i * n + j] -= f * X[k * n + j];
      }
    }
  }
  return true;
}

// Mandel basis tensor B_a (row-major 3x3)
static void mandel_tensor(int a, double B[9]) {
  std::memset(B, 0, 9 * sizeof(double));
  const int i = kPair[a][0], j = kPair[a][1];
  if (i == j) B[i * 3 + i] = 1.0;
  else {
    B[i * 3 + j] = B[j * 3 + i] = 1.0 / std::sqrt(2.0);
  }
}

// row-major 3x3 <-> stored component order
static void rm_to_stored(int kin, const double rm[9], double st[9]) {
  if (kin == KIN_FINITE) {
    for (int c = 0; c < 9; ++c) st[c] = rm[c];
  } else {
    for (int c = 0; c < 6; ++c) st[c] = rm[kPair[c][0] * 3 + kPair[c][1]];
    for (int c = 6; c < 9; ++c) st[c] = 0.0;
  }
}
static void stored_to_rm(int kin, const double st[9], double rm[9]) {
  if (kin == KIN_FINITE) {
    for (int c = 0; c < 9; ++c) rm[c] = st[c];
  } else {
    for (int c = 0; c < 6; ++c) {
      rm[kPair[c][0] * 3 + kPair[c][1]] = st[c];
      rm[kPair[c][1] * 3 + kPair[c][0]] = st[c];
    }
  }
}

template <typename T>
struct Tables {
  void *tw1, *tw2, *tw3, *rtw;
};

struct Ctx {
  int n[3];
  Geom g;
  int kin, prec, mat, ncomp;
  hipStream_t st;
  FftPlan p1, p2, p3;
  Tables<double> td;
  Tables<float> tf;

  // material
  int nphase = 0;
  uint8_t* phase = nullptr;
  double* E64 = nullptr;
  float* E32 = nullptr;
  int32_t* grain = nullptr;
  int ngrain = 0;
  double* grain21 = nullptr;  // [ngrain][21] Mandel upper triangle
  double* grainC = nullptr;   // [ngrain][36]
  double* grainS = nullptr;   // [ngrain][36] inverse
  double lam[kMaxPhases] = {0}, mu[kMaxPhases] = {0};
  double nu = 0.3, lam1 = 0, mu1 = 0;
  double j2_s0 = 0, j2_m = 0, j2_edot0 = 0;

  // workspaces
  void* W = nullptr;  // ncomp x nh complex double
  void *x = nullptr, *r = nullptr, *p = nullptr, *q = nullptr, *b = nullptr, *t64 = nullptr;
  double* sol = nullptr;   // FP64 coefficients of the solution
  double* sol2 = nullptr;  // adjoint solution
  double *fa = nullptr, *fb = nullptr, *fc = nullptr;  // real FP64 fields ncomp x N
  double *state = nullptr, *state_new = nullptr;        // J2 plastic strain (Mandel) 6 x N
  double* tanf = nullptr;                               // J2: 21 x N; neo: 10 x N; SVK: 15 x N (FP64)
  float* tanf32 = nullptr;
  double* partA = nullptr;  // energy partials / general
  double* partB = nullptr;  // update partials
  size_t npart = 0;
  PcgScalars* sc_dev = nullptr;
  PcgScalars* sc_host = nullptr;
  double* dc_dev = nullptr;
  double* mac_dev = nullptr;  // 9 doubles: macro added in the z pass
  double* red_dev = nullptr;  // 128 doubles reduction output
  double* red_host = nullptr;
  int* fail_dev = nullptr;

  // current tangent for apply: 0 elastic, 1 field (after a nonlinear solve)
  int tangent_from_field = 0;

  // optional per-kernel timing of PCG iterations with HIP events
  int prof_on = 0;
  int prof_tag = -1;  // iteration index within the enqueued chunk, -1 = not timed
  std::vector<hipEvent_t> ev_pool, ext_pool;
  std::vector<int> ev_kind, ev_iter, ev_ext;
  double prof_ms[16] = {0};
  long long prof_n[16] = {0};

  // HIP graph of one chunk of PCG iterations, captured on a private stream
  // and replayed on `st`; `chunk_key` holds the launch arguments it was
  // captured with (a solve with other arguments captures again)
  hipStream_t cap_st = nullptr;
  hipGraph_t chunk_graph = nullptr;
  hipGraphExec_t chunk_exec = nullptr;
  std::vector<unsigned char> chunk_key;

  // J2 checkpoints of the last solve (opts.checkpoint): per increment k,
  // the converged coefficients (3 x nh complex) followed by the plastic
  // strain the increment started from (6 x N), and the macro total
  double* ck_buf = nullptr;
  int ck_cap = 0;  // increments ck_buf holds
  int ck_n = 0;    // increments recorded by the last solve
  double ck_dt = 1.0;
  std::vector<std::array<double, 9>> ck_mt;
  double* adj_lam = nullptr;  // J2 adjoint multiplier (Mandel) 6 x N

  // block PCG (dbfft_solve_block): six sets of blk_cap vectors (X R P Q Z P2),
  // per-column macro tensors and mean stresses, block-dot partials
  void* blk = nullptr;
  int blk_cap = 0;
  double* blk_mac = nullptr;
  double* blk_dc = nullptr;
  double* blk_part = nullptr;

  // dbfft_solve_many: the setup arguments a helper context is made from,
  // the device, and the helpers (one per stream, created on first use)
  std::vector<double> setup_params;
  int dev = 0;
  std::vector<dbfft_ctx*> helpers;
  std::vector<hipStream_t> helper_streams;

  // solution state
  bool solved = false;
  int last_mask[9] = {0};
  double EU_st[9] = {0};   // prescribed strain part (stored order)
  double e_st[9] = {0};    // macro unknown as a tensor (stored order)
  double sig_rm[9] = {0}, eps_rm[9] = {0};
  bool use_fused = true;  // opts.fused_cg of the current call
  bool use_graph = true;  // opts.graph of the current call
  bool linear_material() const {
    return mat != DBFFT_MAT_J2VP_CUBIC && mat != DBFFT_MAT_NEOHOOKE && mat != DBFFT_MAT_SVK;
  }
};

enum ProfKind {
  PK_XINV = 0, PK_YINV, PK_ZFUSED, PK_YFWD, PK_XFWD, PK_ALPHA, PK_UPDATE, PK_BETA, PK_PUPDATE, PK_END
};

thread_local LaunchTiming g_launch_timing;

static hipEvent_t pool_event(std::vector<hipEvent_t>& pool, size_t i) {
  while (pool.size() <= i) {
    hipEvent_t e;
    HIPCK(hipEventCreate(&e));
    pool.push_back(e);
  }
  return pool[i];
}

// Marks the start of the kernel of `kind` (PK_END closes the last one): an
// event recorded on the stream brackets the step, and a second pair is left
// for DB_LAUNCH, which records it at the kernel's own start and end.  The
// pair is used when it covered the step's only launch; otherwise the
// bracket (which also holds the gap to the previous kernel) is.
static void prof_mark(Ctx& c, int kind) {
  if (!c.prof_on || c.prof_tag < 0) return;
  LaunchTiming& lt = g_launch_timing;
  if (!c.ev_kind.empty()) c.ev_ext.back() = (lt.consumed && lt.launches == 1) ? 1 : 0;
  lt = LaunchTiming{};
  const size_t i = c.ev_kind.size();
  HIPCK(hipEventRecord(pool_event(c.ev_pool, i), c.st));
  c.ev_kind.push_back(kind);
  c.ev_iter.push_back(c.prof_tag);
  c.ev_ext.push_back(0);
  if (kind < PK_END) {
    lt.start = pool_event(c.ext_pool, 2 * i);
    lt.stop = pool_event(c.ext_pool, 2 * i + 1);
  }
}

// after a stream sync: attribute elapsed times of the first `executed`
// iterations of the chunk
static void prof_collect(Ctx& c, int executed) {
  const size_t n = c.ev_kind.size();
  for (size_t i = 0; i + 1 < n; ++i) {
    const int k = c.ev_kind[i];
    if (k < 0 || k >= PK_END || c.ev_iter[i] >= executed) continue;
    float ms = 0.f;
    if (c.ev_ext[i]) HIPCK(hipEventElapsedTime(&ms, c.ext_pool[2 * i], c.ext_pool[2 * i + 1]));
    else HIPCK(hipEventElapsedTime(&ms, c.ev_pool[i], c.ev_pool[i + 1]));
    c.prof_ms[k] += ms;
    c.prof_n[k] += 1;
  }
  c.ev_kind.clear();
  c.ev_iter.clear();
  c.ev_ext.clear();
  g_launch_timing = LaunchTiming{};
}

static void* dalloc(size_t bytes) {
  void* p = nullptr;
  if (bytes == 0) bytes = 16;
  if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    DB_THROW(DBFFT_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed");
  }
  return p;
}

template <typename T>
static void* upload_table(const std::vector<double>& re, const std::vector<double>& im) {
  std::vector<T> h(2 * re.size());
  for (size_t i = 0; i < re.size(); ++i) {
    h[2 * i] = (T)re[i];
    h[2 * i + 1] = (T)im[i];
  }
  void* d = dalloc(h.size() * sizeof(T));
  HIPCK(hipMemcpy(d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
  return d;
}

static void twiddles(int n, int denom, int count, std::vector<double>& re, std::vector<double>& im) {
  re.resize(count);
  im.resize(count);
  for (int k = 0; k < count; ++k) {
    const double ang = 2.0 * M_PI * (double)k / (double)denom;
    re[k] = std::cos(ang);
    im[k] = -std::sin(ang);
  }
  (void)n;
}

// ------------------------------------------------------------------ tangent args
template <typename T>
static TangentArgs<T> elastic_tangent(Ctx& c);

template <>
TangentArgs<double> elastic_tangent<double>(Ctx& c) {
  TangentArgs<double> t;
  std::memset(&t, 0, sizeof(t));
  t.nphase = c.nphase;
  for (int i = 0; i < kMaxPhases; ++i) {
    t.lam[i] = c.lam[i];
    t.mu[i] = c.mu[i];
  }
  t.lam1 = c.lam1;
  t.mu1 = c.mu1;
  t.phase = c.phase;
  t.grain = c.grain;
  t.grain_table = c.grain21;
  switch (c.mat) {
    case DBFFT_MAT_ISO_PHASE: t.kind = TAN_ISO_PHASE; break;
    case DBFFT_MAT_ISO_FIELD: t.kind = TAN_ISO_FIELD; t.field = c.E64; break;
    case DBFFT_MAT_NEOHOOKE: t.kind = TAN_NEO_FIELD; t.field = c.tanf; break;
    case DBFFT_MAT_SVK: t.kind = TAN_SVK_FIELD; t.field = c.tanf; break;
    case DBFFT_MAT_J2VP_CUBIC:
      if (c.tangent_from_field) {
        t.kind = TAN_ANISO_FIELD;
        t.field = c.tanf;
      } else {
        t.kind = TAN_ANISO_GRAIN;
      }
      break;
    default: t.kind = TAN_ANISO_GRAIN; break;
  }
  return t;
}

template <>
TangentArgs<float> elastic_tangent<float>(Ctx& c) {
  TangentArgs<double> d = elastic_tangent<double>(c);
  TangentArgs<float> t;
  std::memset(&t, 0, sizeof(t));
  t.kind = d.kind;
  t.nphase = d.nphase;
  for (int i = 0; i < kMaxPhases; ++i) {
    t.lam[i] = d.lam[i];
    t.mu[i] = d.mu[i];
  }
  t.lam1 = d.lam1;
  t.mu1 = d.mu1;
  t.phase = d.phase;
  t.grain = d.grain;
  t.grain_table = d.grain_table;
  if (d.kind == TAN_ISO_FIELD) t.field = c.E32;
  else if (d.kind == TAN_ANISO_FIELD || d.kind == TAN_NEO_FIELD || d.kind == TAN_SVK_FIELD) t.field = c.tanf32;
  return t;
}

template <typename T>
static Tables<T>& tables(Ctx& c);
template <>
Tables<double>& tables<double>(Ctx& c) { return c.td; }
template <>
Tables<float>& tables<float>(Ctx& c) { return c.tf; }

static StridedGeom xgeom(const Ctx& c) {
  StridedGeom s;
  s.nline = c.n[0];
  s.lstride = (long long)c.n[1] * c.g.nh3;
  s.ostride = c.g.nh3;
  s.nother = c.n[1];
  s.ncols = c.g.nh3;
  s.cstride_in = c.g.nh;
  s.cstride_out = c.g.nh;
  return s;
}
static StridedGeom ygeom(const Ctx& c) {
  StridedGeom s;
  s.nline = c.n[1];
  s.lstride = c.g.nh3;
  s.ostride = (long long)c.n[1] * c.g.nh3;
  s.nother = c.n[0];
  s.ncols = c.g.nh3;
  s.cstride_in = c.g.nh;
  s.cstride_out = c.g.nh;
  return s;
}

// ------------------------------------------------------------------ operator pieces
// K a: x inverse + gradient -> y inverse -> z fused tangent -> y forward -> x forward + divergence
// (whose first block computes alpha when `at` names the PCG state)
template <typename T>
static void apply_K(Ctx& c, const void* a, void* out, const double* macro_dev, const double* macro_add,
                    const TangentArgs<T>& tan, double* energy_partials, double* dc_out, const int* stop,
                    const AlphaTask& at = AlphaTask()) {
  Tables<T>& tb = tables<T>(c);
  const StridedGeom sx = xgeom(c), sy = ygeom(c);
  const int gm = (c.kin == KIN_SMALL) ? SP_GRAD_SMALL : SP_GRAD_FINITE;
  const int dm = (c.kin == KIN_SMALL) ? SP_DIV_SMALL : SP_DIV_FINITE;
  prof_mark(c, PK_XINV);
  launch_strided<T>(gm, a, c.W, 0, sx, c.g, c.p1, tb.tw1, +1, nullptr, c.st, stop);
  prof_mark(c, PK_YINV);
  launch_strided<T>(SP_PLAIN, c.W, c.W, c.ncomp, sy, c.g, c.p2, tb.tw2, +1, nullptr, c.st, stop);
  int nb = 0;
  prof_mark(c, PK_ZFUSED);
  launch_line<T>(LP_FUSED, c.kin, c.W, c.W, c.g, c.p3, tb.tw3, tb.rtw, tan, macro_dev, macro_add, energy_partials,
                 c.ncomp, c.st, &nb, stop);
  prof_mark(c, PK_YFWD);
  launch_strided<T>(SP_PLAIN, c.W, c.W, c.ncomp, sy, c.g, c.p2, tb.tw2, -1, nullptr, c.st, stop);
  prof_mark(c, PK_XFWD);
  launch_strided<T>(dm, c.W, out, 0, sx, c.g, c.p1, tb.tw1, -1, dc_out, c.st, stop, at);
}

template <typename T>
static int energy_blocks(Ctx& c, int tan_kind) {
  return fused_line_blocks(c.g, c.ncomp, (int)(2 * sizeof(T)), tan_kind);
}

// K [0; E] (stress of a uniform strain E): -> out (3 comps), dc
template <typename T>
static void apply_const(Ctx& c, void* out, const double* macro_add, const TangentArgs<T>& tan, double* dc_out) {
  Tables<T>& tb = tables<T>(c);
  const StridedGeom sx = xgeom(c), sy = ygeom(c);
  const int dm = (c.kin == KIN_SMALL) ? SP_DIV_SMALL : SP_DIV_FINITE;
  launch_line<T>(LP_CONST, c.kin, nullptr, c.W, c.g, c.p3, tb.tw3, tb.rtw, tan, nullptr, macro_add, nullptr,
                 c.ncomp, c.st, nullptr, nullptr);
  launch_strided<T>(SP_PLAIN, c.W, c.W, c.ncomp, sy, c.g, c.p2, tb.tw2, -1, nullptr, c.st, nullptr);
  launch_strided<T>(dm, c.W, out, 0, sx, c.g, c.p1, tb.tw1, -1, dc_out, c.st, nullptr);
}

// real strain (or H) field of coefficients a (FP64) plus uniform macro part
static void strain_field(Ctx& c, const void* a, const double* macro_add, double* out, int with_tangent = 0) {
  Tables<double>& tb = c.td;
  const StridedGeom sx = xgeom(c), sy = ygeom(c);
  const int gm = (c.kin == KIN_SMALL) ? SP_GRAD_SMALL : SP_GRAD_FINITE;
  launch_strided<double>(gm, a, c.W, 0, sx, c.g, c.p1, tb.tw1, +1, nullptr, c.st, nullptr);
  launch_strided<double>(SP_PLAIN, c.W, c.W, c.ncomp, sy, c.g, c.p2, tb.tw2, +1, nullptr, c.st, nullptr);
  TangentArgs<double> tan = elastic_tangent<double>(c);
  launch_line<double>(with_tangent ? LP_STRESS : LP_C2R, c.kin, c.W, out, c.g, c.p3, tb.tw3, tb.rtw, tan, nullptr,
                      macro_add, nullptr, c.ncomp, c.st, nullptr, nullptr);
}

// residual i xi_j F[sigma]_ij / N of a real FP64 stress field -> out (FP64, = -K-form), dc
static void stress_residual(Ctx& c, const double* sig, void* out, double* dc_out) {
  Tables<double>& tb = c.td;
  const StridedGeom sx = xgeom(c), sy = ygeom(c);
  const int dm = (c.kin == KIN_SMALL) ? SP_DIV_SMALL : SP_DIV_FINITE;
  TangentArgs<double> tan = elastic_tangent<double>(c);
  launch_line<double>(LP_R2C, c.kin, sig, c.W, c.g, c.p3, tb.tw3, tb.rtw, tan, nullptr, nullptr, nullptr, c.ncomp,
                      c.st, nullptr, nullptr);
  launch_strided<double>(SP_PLAIN, c.W, c.W, c.ncomp, sy, c.g, c.p2, tb.tw2, -1, nullptr, c.st, nullptr);
  launch_strided<double>(dm, c.W, out, 0, sx, c.g, c.p1, tb.tw1, -1, dc_out, c.st, nullptr);
  // out holds -i xi_j s_ij; the residual is its negative
  launch_axpby<double>(out, out, 0.0, -1.0, 6 * c.g.nh, c.st);
}

static double dot64(Ctx& c, const void* u, const void* v) {
  const int nb = pcg_block_count(c.g);
  launch_dot_w(u, v, 0, c.g, c.partB, nb, c.st);
  launch_reduce(c.partB, nb, 1, c.red_dev, c.st);
  HIPCK(hipMemcpyAsync(c.red_host, c.red_dev, sizeof(double), hipMemcpyDeviceToHost, c.st));
  HIPCK(hipStreamSynchronize(c.st));
  return c.red_host[0];
}

static void read_dc(Ctx& c, double dc_st[9]) {
  HIPCK(hipMemcpyAsync(c.red_host, c.dc_dev, 9 * sizeof(double), hipMemcpyDeviceToHost, c.st));
  HIPCK(hipStreamSynchronize(c.st));
  for (int i = 0; i < 9; ++i) dc_st[i] = (i < c.ncomp) ? c.red_host[i] : 0.0;
}

static void set_macro(Ctx& c, const double st9[9]) {
  double h[9];
  for (int i = 0; i < 9; ++i) h[i] = st9[i];
  HIPCK(hipMemcpyAsync(c.mac_dev, h, 9 * sizeof(double), hipMemcpyHostToDevice, c.st));
  HIPCK(hipStreamSynchronize(c.st));
}

static double frob_stored(int kin, const double t[9]) {
  double s = 0.0;
  if (kin == KIN_SMALL) {
    for (int i = 0; i < 3; ++i) s += t[i] * t[i];
    for (int i = 3; i < 6; ++i) s += 2.0 * t[i] * t[i];
  } else {
    for (int i = 0; i < 9; ++i) s += t[i] * t[i];
  }
  return std::sqrt(s);
}

// ------------------------------------------------------------------ macro basis and preconditioner
struct MacroSet {
  int nS = 0;
  int idx[kMaxMacro];
  double bst[kMaxMacro][9];  // basis tensors in stored order
};

static MacroSet macro_set(const Ctx& c, const int mask[9]) {
  MacroSet m;
  if (c.kin == KIN_SMALL) {
    for (int a = 0; a < 6; ++a) {
      if (mask[kPair[a][0] * 3 + kPair[a][1]]) {
        double B[9], s[9];
        mandel_tensor(a, B);
        rm_to_stored(KIN_SMALL, B, s);
        m.idx[m.nS] = a;
        for (int k = 0; k < 9; ++k) m.bst[m.nS][k] = s[k];
        m.nS++;
      }
    }
  } else {
    for (int a = 0; a < 9; ++a) {
      if (mask[a]) {
        m.idx[m.nS] = a;
        for (int k = 0; k < 9; ++k) m.bst[m.nS][k] = (k == a) ? 1.0 : 0.0;
        m.nS++;
      }
    }
  }
  return m;
}

// contraction B : t with t in stored order
static double bdot(int kin, const double B[9], const double t[9]) {
  double s = 0.0;
  for (int k = 0; k < 9; ++k) s += B[k] * t[k] * ((kin == KIN_SMALL && k >= 3 && k < 6) ? 2.0 : 1.0);
  return s;
}

// mean tangent -> 4th order C[i][j][k][l] (FP64)
static void mean_tangent(Ctx& c, double C4[81]) {
  TangentArgs<double> tan = elastic_tangent<double>(c);
  const int nb = tangent_mean_block_count(c.g);
  const int nv = tangent_mean_nvals(c.kin);
  launch_tangent_mean<double>(tan, c.kin, c.g, c.partA, nb, c.st);
  launch_reduce(c.partA, nb, nv, c.red_dev, c.st);
  HIPCK(hipMemcpyAsync(c.red_host, c.red_dev, nv * sizeof(double), hipMemcpyDeviceToHost, c.st));
  HIPCK(hipStreamSynchronize(c.st));
  const double inv = c.g.inv_nvox;
  if (c.kin == KIN_SMALL) {
    double M[6][6];
    int idx = 0;
    for (int a = 0; a < 6; ++a)
      for (int b = a; b < 6; ++b) {
        M[a][b] = M[b][a] = c.red_host[idx++] * inv;
      }
    double B[6][9];
    for (int a = 0; a < 6; ++a) mandel_tensor(a, B[a]);
    for (int i = 0; i < 81; ++i) C4[i] = 0.0;
    for (int a = 0; a < 6; ++a)
      for (int b = 0; b < 6; ++b) {
        if (M[a][b] == 0.0) continue;
        for (int ij = 0; ij < 9; ++ij)
          for (int kl = 0; kl < 9; ++kl) C4[ij * 9 + kl] += B[a][ij] * M[a][b] * B[b][kl];
      }
  } else {
    for (int i = 0; i < 81; ++i) C4[i] = c.red_host[i] * inv;
  }
}

static void build_precond(const Ctx& c, const double C4[81], const MacroSet& ms, PrecondArgs& pa, PcgConst& pc) {
  // q = (j, l) pairs and m = (i, k) pairs in storage 00 11 22 12 02 01
  auto C = [&](int i, int j, int k, int l) { return C4[((i * 3 + j) * 3 + k) * 3 + l]; };
  for (int q = 0; q < 6; ++q) {
    const int j = kPair[q][0], l = kPair[q][1];
    for (int m = 0; m < 6; ++m) {
      const int i = kPair[m][0], k = kPair[m][1];
      double v = (j == l) ? C(i, j, k, j) : C(i, j, k, l) + C(i, l, k, j);
      if (i != k) {
        // symmetric part of A_ik
        const double v2 = (j == l) ? C(k, j, i, j) : C(k, j, i, l) + C(k, l, i, j);
        v = 0.5 * (v + v2);
      }
      pa.G[q][m] = v;
    }
  }
  pc.nmacro = ms.nS;
  pc.ncomp = c.ncomp;
  for (int a = 0; a < kMaxMacro; ++a)
    for (int k = 0; k < 9; ++k) pc.basis[a][k] = (a < ms.nS) ? ms.bst[a][k] : 0.0;
  for (int a = 0; a < kMaxMacro; ++a)
    for (int b = 0; b < kMaxMacro; ++b) pc.Me[a][b] = 0.0;
  if (ms.nS > 0) {
    // Cee_ab = B_a : C : B_b (B in row-major)
    std::vector<double> Cee(ms.nS * ms.nS), inv;
    for (int a = 0; a < ms.nS; ++a)
      for (int b = 0; b < ms.nS; ++b) {
        double Ba[9], Bb[9];
        stored_to_rm(c.kin, ms.bst[a], Ba);
        stored_to_rm(c.kin, ms.bst[b], Bb);
        double s = 0.0;
        for (int ij = 0; ij < 9; ++ij)
          for (int kl = 0; kl < 9; ++kl) s += Ba[ij] * C4[ij * 9 + kl] * Bb[kl];
        Cee[a * ms.nS + b] = s;
      }
    if (!small_inverse(Cee, ms.nS, inv)) DB_THROW(DBFFT_EBREAKDOWN, "singular mean stiffness on the stress-controlled set");
    for (int a = 0; a < ms.nS; ++a)
      for (int b = 0; b < ms.nS; ++b) pc.Me[a][b] = inv[a * ms.nS + b];
  }
}

// ------------------------------------------------------------------ PCG driver
struct PcgOut {
  int iters;
  int status;  // 1 conv, 2 breakdown, 3 cap
  double eq, ld;
  double sig[9];
  double xe[kMaxMacro];
};

// Sets x = 0, the scalars (<sigma> of the field that produced b, macro
// residual), p = M r and <r, M r>; b is in r (precision T).  Synchronizes.
template <typename T>
static void pcg_begin(Ctx& c, const PrecondArgs& pa, const PcgConst& pc, void* x, void* r, void* p,
                      const double sig0[9], const double re0[kMaxMacro]) {
  const size_t vbytes = 3 * (size_t)c.g.nh * 2 * sizeof(T);
  HIPCK(hipMemsetAsync(x, 0, vbytes, c.st));
  PcgScalars& h = *c.sc_host;
  std::memset(&h, 0, sizeof(h));
  for (int i = 0; i < 9; ++i) h.sig[i] = sig0[i];
  for (int a = 0; a < kMaxMacro; ++a) h.re[a] = re0[a];
  HIPCK(hipMemcpyAsync(c.sc_dev, c.sc_host, sizeof(PcgScalars), hipMemcpyHostToDevice, c.st));
  const int nb = pcg_block_count(c.g);
  launch_precond_init<T>(p, r, pa, c.g, c.partB, nb, c.st);
  launch_pcg_beta(c.sc_dev, c.partB, nb, pc, 1, c.st);
  HIPCK(hipMemcpyAsync(c.sc_host, c.sc_dev, sizeof(PcgScalars), hipMemcpyDeviceToHost, c.st));
  HIPCK(hipStreamSynchronize(c.st));
}

// Goes on with the direction p after the residual in r was replaced by a
// recomputed one (precision T): x = 0 for the next segment's step sum,
// the scalars take the recomputed <sigma> and macro residual, r is
// projected onto Hermitian pairs, and p = M r + beta p with
// beta = <r, M r> / rho_prev (rho_prev: the <r, M r> the direction was last
// formed with).  The iteration counter restarts at 0.  Synchronizes.
template <typename T>
static void pcg_resume(Ctx& c, const PrecondArgs& pa, const PcgConst& pc, void* x, void* r, void* p,
                       const double sig[9], const double re[kMaxMacro], double rho_prev) {
  const size_t vbytes = 3 * (size_t)c.g.nh * 2 * sizeof(T);
  HIPCK(hipMemsetAsync(x, 0, vbytes, c.st));
  PcgScalars& h = *c.sc_host;
  for (int i = 0; i < 9; ++i) h.sig[i] = sig[i];
  for (int a = 0; a < kMaxMacro; ++a) {
    h.re[a] = re[a];
    h.xe[a] = 0.0;
  }
  h.rz = rho_prev;
  h.iter = 0;
  h.converged = 0;
  h.pending = 0;
  HIPCK(hipMemcpyAsync(c.sc_dev, c.sc_host, sizeof(PcgScalars), hipMemcpyHostToDevice, c.st));
  const int nb = pcg_block_count(c.g);
  launch_precond_dots<T>(r, pa, c.g, c.partB, nb, c.st);
  launch_pcg_beta(c.sc_dev, c.partB, nb, pc, 2, c.st);
  launch_pcg_pupdate<T>(p, r, c.sc_dev, pa, c.g, nb, c.st);
  HIPCK(hipMemcpyAsync(c.sc_host, c.sc_dev, sizeof(PcgScalars), hipMemcpyDeviceToHost, c.st));
  HIPCK(hipStreamSynchronize(c.st));
}

static PcgOut pcg_result(Ctx& c) {
  const PcgScalars& h = *c.sc_host;
  if (g_verbose)
    std::fprintf(stderr, "[dbfft] pcg: iters %d status %d eq %.3e load %.3e rz %.3e pq %.3e\n", h.iter, h.converged,
                 h.eq_res, h.load_res, h.rz, h.pq);
  PcgOut o;
  o.iters = h.iter;
  o.status = h.converged;
  o.eq = h.eq_res;
  o.ld = h.load_res;
  for (int i = 0; i < 9; ++i) o.sig[i] = h.sig[i];
  for (int a = 0; a < kMaxMacro; ++a) o.xe[a] = h.xe[a];
  return o;
}

// The fused iteration needs the register-FFT x pass (n1 a power of two from
// 8 to 256), n2 even (Hermitian partner lines in the same block) and small
// strains; opts.fused_cg = 0 selects the separate vector kernels.
static bool fused_cg(const Ctx& c) {
  return c.use_fused && c.kin == KIN_SMALL && fast_strided_supported(c.n[0]) && c.n[1] % 2 == 0;
}

// Launch arguments of one PCG chunk, byte for byte: a chunk graph captured
// with an equal key replays exactly the launches the eager loop would make.
template <typename T>
static std::vector<unsigned char> chunk_key(const Ctx& c, const TangentArgs<T>& tan, const PrecondArgs& pa,
                                            const PcgConst& pc, const void* x, const void* r, const void* p,
                                            const void* q, int check_every) {
  std::vector<unsigned char> k;
  auto put = [&](const void* v, size_t n) {
    const unsigned char* b = static_cast<const unsigned char*>(v);
    k.insert(k.end(), b, b + n);
  };
  const int head[3] = {(int)sizeof(T), check_every, fused_cg(c) ? 1 : 0};
  const void* vec[4] = {x, r, p, q};
  put(head, sizeof(head));
  put(vec, sizeof(vec));
  put(&tan, sizeof(tan));
  put(&pa, sizeof(pa));
  put(&pc, sizeof(pc));
  return k;
}

// Solves K x = b with b in r (precision T); x is overwritten (starts at 0).
// The iterations are enqueued in chunks of `check_every`, each followed by
// a read of the device scalars.  The first chunk is launched eagerly; a
// solve that needs more captures one chunk in a HIP graph (unless kernel
// timing is on) and replays it, which takes the per-launch host cost out of
// every later chunk.
// rho_prev > 0: go on with the direction in p (pcg_resume) instead of
// starting from p = M r.
template <typename T>
static PcgOut run_pcg(Ctx& c, const TangentArgs<T>& tan, const PrecondArgs& pa, const PcgConst& pc, void* x, void* r,
                      void* p, void* q, const double sig0[9], const double re0[kMaxMacro], int check_every,
                      double rho_prev = 0.0) {
  if (rho_prev > 0.0) pcg_resume<T>(c, pa, pc, x, r, p, sig0, re0, rho_prev);
  else pcg_begin<T>(c, pa, pc, x, r, p, sig0, re0);
  const int nb = pcg_block_count(c.g);
  const int neb = energy_blocks<T>(c, tan.kind);
  const double* pmac = reinterpret_cast<const double*>(reinterpret_cast<const char*>(c.sc_dev) + offsetof(PcgScalars, pmac));
  const int* stop = reinterpret_cast<const int*>(reinterpret_cast<const char*>(c.sc_dev) + offsetof(PcgScalars, converged));
  if (check_every < 1) check_every = 1;
  const bool fused = fused_cg(c);
  // one chunk of iterations on stream s (c.st itself, or the capture stream)
  // Kernel timing samples the middle iteration of every chunk (the events
  // a launch records cost the stream a few microseconds each; the kernels of
  // every iteration are the same work).
  const int sample = check_every / 2;
  auto enqueue_chunk = [&](hipStream_t s) {
    const hipStream_t st_saved = c.st;
    c.st = s;
    for (int k = 0; k < check_every; ++k) {
      if (k == sample + 1) {
        c.prof_tag = sample;
        prof_mark(c, PK_END);
      }
      c.prof_tag = (k == sample) ? k : -1;
      if (fused) {
        // gradient | y | z (+ <p, K p> partials) | y (its first block: alpha)
        // | divergence with r -= alpha q and the Hermitian planes | beta (+
        // macroscopic step) | x += alpha p, next p
        Tables<T>& tb = tables<T>(c);
        const StridedGeom sx = xgeom(c), sy = ygeom(c);
        prof_mark(c, PK_XINV);
        launch_strided<T>(SP_GRAD_SMALL, p, c.W, 0, sx, c.g, c.p1, tb.tw1, +1, nullptr, c.st, stop);
        prof_mark(c, PK_YINV);
        launch_strided<T>(SP_PLAIN, c.W, c.W, c.ncomp, sy, c.g, c.p2, tb.tw2, +1, nullptr, c.st, stop);
        prof_mark(c, PK_ZFUSED);
        launch_line<T>(LP_FUSED, c.kin, c.W, c.W, c.g, c.p3, tb.tw3, tb.rtw, tan, pmac, nullptr, c.partA, c.ncomp,
                       c.st, nullptr, stop);
        AlphaTask at;
        at.sc = c.sc_dev;
        at.eparts = c.partA;
        at.neparts = neb;
        prof_mark(c, PK_YFWD);
        launch_strided<T>(SP_PLAIN, c.W, c.W, c.ncomp, sy, c.g, c.p2, tb.tw2, -1, nullptr, c.st, stop, at);
        prof_mark(c, PK_XFWD);
        const int nd = launch_div_update_fast<T>(c.W, r, sx, c.g, tb.tw1, c.sc_dev, pa, c.dc_dev, c.partB, c.st);
        prof_mark(c, PK_BETA);
        launch_pcg_beta_step(c.sc_dev, c.partB, nd, c.dc_dev, pc, c.st);
        prof_mark(c, PK_PUPDATE);
        launch_pcg_xp<T>(x, p, r, c.sc_dev, pa, c.g, nb, c.st);
        continue;
      }
      // K p (the first block of its x forward pass: alpha) | r -= alpha q |
      // beta (+ macroscopic step) | x += alpha p, next p
      AlphaTask at;
      at.sc = c.sc_dev;
      at.eparts = c.partA;
      at.neparts = neb;
      apply_K<T>(c, p, q, pmac, nullptr, tan, c.partA, c.dc_dev, stop, at);
      prof_mark(c, PK_UPDATE);
      launch_pcg_update<T>(nullptr, r, p, q, c.sc_dev, pa, c.g, c.partB, nb, c.st);
      prof_mark(c, PK_BETA);
      launch_pcg_beta_step(c.sc_dev, c.partB, nb, c.dc_dev, pc, c.st);
      prof_mark(c, PK_PUPDATE);
      launch_pcg_xp<T>(x, p, r, c.sc_dev, pa, c.g, nb, c.st);
    }
    if (sample == check_every - 1) {
      c.prof_tag = sample;
      prof_mark(c, PK_END);
    }
    c.prof_tag = -1;
    c.st = st_saved;
  };
  bool first = true;
  while (!c.sc_host->converged) {
    const int iter0 = c.sc_host->iter;
    if (!first && !c.prof_on && c.use_graph) {
      std::vector<unsigned char> key = chunk_key<T>(c, tan, pa, pc, x, r, p, q, check_every);
      if (c.chunk_exec == nullptr || key != c.chunk_key) {
        if (c.chunk_exec) HIPCK(hipGraphExecDestroy(c.chunk_exec));
        if (c.chunk_graph) HIPCK(hipGraphDestroy(c.chunk_graph));
        c.chunk_exec = nullptr;
        c.chunk_graph = nullptr;
        c.chunk_key.clear();
        if (c.cap_st == nullptr) HIPCK(hipStreamCreateWithFlags(&c.cap_st, hipStreamNonBlocking));
        HIPCK(hipStreamBeginCapture(c.cap_st, hipStreamCaptureModeThreadLocal));
        enqueue_chunk(c.cap_st);
        HIPCK(hipStreamEndCapture(c.cap_st, &c.chunk_graph));
        HIPCK(hipGraphInstantiate(&c.chunk_exec, c.chunk_graph, nullptr, nullptr, 0));
        c.chunk_key.swap(key);
        if (g_verbose) std::fprintf(stderr, "[dbfft] pcg: captured a graph of %d iterations\n", check_every);
      }
      HIPCK(hipGraphLaunch(c.chunk_exec, c.st));
    } else {
      enqueue_chunk(c.st);
    }
    first = false;
    HIPCK(hipGetLastError());
    HIPCK(hipMemcpyAsync(c.sc_host, c.sc_dev, sizeof(PcgScalars), hipMemcpyDeviceToHost, c.st));
    HIPCK(hipStreamSynchronize(c.st));
    if (c.prof_on) prof_collect(c, c.sc_host->iter - iter0 - (c.sc_host->converged ? 1 : 0));
  }
  return pcg_result(c);
}

// ------------------------------------------------------------------ linear solve
struct LinOut {
  int iters = 0, refine = 0, status = DBFFT_OK;
  double eq = 0, ld = 0;
  double sig_st[9] = {0};
  double e_coef[kMaxMacro] = {0};
};

static int pcg_status(int s) {
  if (s == 1) return DBFFT_OK;
  if (s == 2) return DBFFT_EBREAKDOWN;
  return DBFFT_ENOTCONV;
}

// Solves the linear problem with prescribed strain EU (stored) and stress
// row sbar (over the macro set) into sol_out (FP64 coefficients).
// PCG solve of K [x; e] = [c.b; re0] with the current tangent: c.b holds
// the FP64 right-hand side, dc0 the <sigma> of the field that produced it.
// FP64 directly; FP32_MIXED as FP32 inner solves with FP64 corrections.
// scale > 0 replaces ||<sigma>|| in the residual test.
static LinOut linear_solve_b(Ctx& c, const MacroSet& ms, const double dc0[9], const double re0[kMaxMacro],
                             const dbfft_opts& o, double* sol_out, double scale = 0.0) {
  LinOut out;
  double C4[81];
  mean_tangent(c, C4);
  PrecondArgs pa{};
  PcgConst pc{};
  std::memset(&pc, 0, sizeof(pc));
  build_precond(c, C4, ms, pa, pc);
  pc.tol = o.tol;
  pc.tol_load = o.tol_load;
  pc.max_iter = o.max_iter;
  pc.scale = scale;
  const size_t v64 = 3 * (size_t)c.g.nh * 2 * sizeof(double);
  TangentArgs<double> tan64 = elastic_tangent<double>(c);

  if (c.prec == DBFFT_FP64) {
    HIPCK(hipMemcpyAsync(c.r, c.b, v64, hipMemcpyDeviceToDevice, c.st));
    PcgOut po = run_pcg<double>(c, tan64, pa, pc, sol_out, c.r, c.p, c.q, dc0, re0, o.check_every);
    out.iters = po.iters;
    out.status = pcg_status(po.status);
    out.eq = po.eq;
    out.ld = po.ld;
    for (int i = 0; i < 9; ++i) out.sig_st[i] = po.sig[i];
    for (int a = 0; a < kMaxMacro; ++a) out.e_coef[a] = po.xe[a];
    return out;
  }

  // FP32 PCG with FP64 residual replacement: the FP32 iteration runs until
  // its recursively updated residual has dropped by inner_tol; then the
  // step sum joins the FP64 solution, the FP64 residual b - K64 x replaces
  // the FP32 one, and the iteration goes on with the same direction
  // (beta from the replaced residual), so the Krylov space built so far is
  // kept.  A segment that stops at its first test has no direction yet and
  // starts from p = M r.
  TangentArgs<float> tan32 = elastic_tangent<float>(c);
  HIPCK(hipMemsetAsync(sol_out, 0, v64, c.st));
  double e[kMaxMacro] = {0};
  double sig[9], re[kMaxMacro];
  for (int i = 0; i < 9; ++i) sig[i] = dc0[i];
  for (int a = 0; a < kMaxMacro; ++a) re[a] = re0[a];
  void* r64 = c.t64;
  HIPCK(hipMemcpyAsync(r64, c.b, v64, hipMemcpyDeviceToDevice, c.st));
  double rho_prev = 0.0, rec_eq = 0.0, rec_ld = 0.0;
  for (int it = 0;; ++it) {
    if (it > 0) {
      // r64 = b - K64 [x; e]
      double mt[9] = {0};
      for (int a = 0; a < ms.nS; ++a)
        for (int k = 0; k < 9; ++k) mt[k] += e[a] * ms.bst[a][k];
      set_macro(c, mt);
      apply_K<double>(c, sol_out, r64, c.mac_dev, nullptr, tan64, c.partA, c.dc_dev, nullptr);
      launch_axpby<double>(r64, c.b, 1.0, -1.0, 6 * c.g.nh, c.st);
      double dcx[9];
      read_dc(c, dcx);
      for (int i = 0; i < 9; ++i) sig[i] = dc0[i] + dcx[i];
      for (int a = 0; a < ms.nS; ++a) re[a] = re0[a] - bdot(c.kin, ms.bst[a], dcx);
    }
    const double nrm = scale > 0.0 ? scale : frob_stored(c.kin, sig);
    const double ra = std::sqrt(std::max(dot64(c, r64, r64), 0.0));
    double rl = 0.0;
    for (int a = 0; a < ms.nS; ++a) rl += re[a] * re[a];
    rl = std::sqrt(rl);
    const double eq = nrm > 0 ? ra / nrm : (ra == 0 ? 0.0 : INFINITY);
    const double ld = nrm > 0 ? rl / nrm : (rl == 0 ? 0.0 : INFINITY);
    // The direction is kept only while the FP32 recursion still tracks the
    // true residual (within a factor of 10 at the segment's end); past that
    // the old direction no longer fits the replaced residual, and the next
    // segment starts from p = M r.
    if (rho_prev > 0.0 && (eq > 10.0 * rec_eq || ld > 10.0 * std::max(rec_ld, 0.1 * o.tol_load))) rho_prev = 0.0;
    out.eq = eq;
    out.ld = ld;
    for (int i = 0; i < 9; ++i) out.sig_st[i] = sig[i];
    for (int a = 0; a < kMaxMacro; ++a) out.e_coef[a] = e[a];
    if (eq < o.tol && ld < o.tol_load) {
      out.status = DBFFT_OK;
      break;
    }
    if (it >= o.max_refine || out.iters >= o.max_iter) {
      out.status = DBFFT_ENOTCONV;
      break;
    }
    PcgConst pci = pc;
    pci.tol = std::max(eq * o.inner_tol, 0.5 * o.tol);
    pci.tol_load = std::max(ld * o.inner_tol, 0.5 * o.tol_load);
    pci.max_iter = std::max(1, o.max_iter - out.iters);
    launch_convert<double, float>(c.r, r64, 6 * c.g.nh, c.st);
    PcgOut po = run_pcg<float>(c, tan32, pa, pci, c.x, c.r, c.p, c.q, sig, re, o.check_every, rho_prev);
    out.iters += po.iters;
    out.refine += 1;
    if (po.status == 2) {
      out.status = DBFFT_EBREAKDOWN;
      break;
    }
    // <r, M r> the last direction was formed with: rz_(k+1) / beta_(k+1)
    const PcgScalars& hs = *c.sc_host;
    rho_prev = (po.status == 1 && hs.beta > 0.0 && hs.rz > 0.0) ? hs.rz / hs.beta : 0.0;
    rec_eq = po.eq;
    rec_ld = po.ld;
    // sol += delta
    launch_convert<float, double>(c.q, c.x, 6 * c.g.nh, c.st);
    launch_axpby<double>(sol_out, c.q, 1.0, 1.0, 6 * c.g.nh, c.st);
    for (int a = 0; a < ms.nS; ++a) e[a] += po.xe[a];
  }
  return out;
}

// linear cell problem with prescribed strain EU and stress sbar on S
static LinOut linear_solve(Ctx& c, const double EU[9], const MacroSet& ms, const double sbar[kMaxMacro],
                           const dbfft_opts& o, double* sol_out) {
  // right-hand side in FP64: b = -K[0; EU], b_e = sbar - B:<C:EU>
  TangentArgs<double> tan64 = elastic_tangent<double>(c);
  set_macro(c, EU);
  apply_const<double>(c, c.b, c.mac_dev, tan64, c.dc_dev);
  launch_axpby<double>(c.b, c.b, 0.0, -1.0, 6 * c.g.nh, c.st);
  double dc0[9];
  read_dc(c, dc0);
  double re0[kMaxMacro] = {0};
  for (int a = 0; a < ms.nS; ++a) re0[a] = sbar[a] - bdot(c.kin, ms.bst[a], dc0);
  return linear_solve_b(c, ms, dc0, re0, o, sol_out);
}

// true residuals and <sigma> of coefficients sol (FP64) with macro total mt (stored)
static void evaluate_linear(Ctx& c, const double* sol, const double mt[9], const MacroSet& ms,
                            const double sbar[kMaxMacro], double sig_st[9], double& eq, double& ld) {
  TangentArgs<double> tan64 = elastic_tangent<double>(c);
  set_macro(c, mt);
  apply_K<double>(c, sol, c.t64, c.mac_dev, nullptr, tan64, c.partA, c.dc_dev, nullptr);
  read_dc(c, sig_st);
  const double ra = std::sqrt(std::max(dot64(c, c.t64, c.t64), 0.0));
  double rl = 0.0;
  for (int a = 0; a < ms.nS; ++a) {
    const double d = sbar[a] - bdot(c.kin, ms.bst[a], sig_st);
    rl += d * d;
  }
  rl = std::sqrt(rl);
  const double nrm = frob_stored(c.kin, sig_st);
  eq = nrm > 0 ? ra / nrm : 0.0;
  ld = nrm > 0 ? rl / nrm : 0.0;
}

// ------------------------------------------------------------------ block PCG
// Several loads of one linear cell (one stress mask) solved in one block
// Krylov space of the preconditioned operator (FP64).  P is a block of
// K-conjugate directions, Q = K P:
//   alpha = (P^T Q)^-1 P^T R,  X += P alpha,  R -= Q alpha,
//   beta = -(P^T Q)^-1 Q^T Z with Z = M R,  next P = orthonormal basis of Z + P beta,
// with the real inner product on the half spectrum plus the Euclidean one on
// the macro block.  Converged columns leave the block; the orthonormal basis
// comes from a Cholesky factorization of the Gram matrix with diagonal
// pivoting that drops dependent directions.  Block inner products and
// combinations are vector kernels; the small matrices are solved here.

// Cholesky of an n x n SPD matrix (row-major), lower factor in L; false if not SPD
static bool chol(const std::vector<double>& A, int n, std::vector<double>& L) {
  L.assign(n * n, 0.0);
  for (int j = 0; j < n; ++j) {
    double d = A[j * n + j];
    for (int k = 0; k < j; ++k) d -= L[j * n + k] * L[j * n + k];
    if (!(d > 0.0)) return false;
    L[j * n + j] = std::sqrt(d);
    for (int i = j + 1; i < n; ++i) {
      double v = A[i * n + j];
      for (int k = 0; k < j; ++k) v -= L[i * n + k] * L[j * n + k];
      L[i * n + j] = v / L[j * n + j];
    }
  }
  return true;
}
// X = A^-1 B for A = L L^T (B: n x m, row-major)
static std::vector<double> chol_solve(const std::vector<double>& L, int n, const std::vector<double>& B, int m) {
  std::vector<double> X(B);
  for (int c = 0; c < m; ++c) {
    for (int i = 0; i < n; ++i) {
      double v = X[i * m + c];
      for (int k = 0; k < i; ++k) v -= L[i * n + k] * X[k * m + c];
      X[i * m + c] = v / L[i * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {
      double v = X[i * m + c];
      for (int k = i + 1; k < n; ++k) v -= L[k * n + i] * X[k * m + c];
      X[i * m + c] = v / L[i * n + i];
    }
  }
  return X;
}

struct BlockVec {
  void* a = nullptr;              // device half-spectrum coefficients
  double e[kMaxMacro] = {0};      // macro block
};

// inner products of the vectors of two lists: out[i * |B| + j]
static std::vector<double> blk_dot(Ctx& c, const std::vector<BlockVec*>& A, const std::vector<BlockVec*>& B, int nS) {
  const int na = (int)A.size(), nb = (int)B.size();
  BlockVecs va{}, vb{};
  for (int i = 0; i < na; ++i) va.v[i] = A[i]->a;
  for (int j = 0; j < nb; ++j) vb.v[j] = B[j]->a;
  const int nblk = pcg_block_count(c.g);
  launch_block_dot(va, vb, na, nb, c.g, c.blk_part, nblk, c.st);
  launch_reduce(c.blk_part, nblk, na * nb, c.red_dev, c.st);
  HIPCK(hipMemcpyAsync(c.red_host, c.red_dev, na * nb * sizeof(double), hipMemcpyDeviceToHost, c.st));
  HIPCK(hipStreamSynchronize(c.st));
  std::vector<double> out(na * nb);
  for (int i = 0; i < na; ++i)
    for (int j = 0; j < nb; ++j) {
      double v = c.red_host[i * nb + j];
      for (int a = 0; a < nS; ++a) v += A[i]->e[a] * B[j]->e[a];
      out[i * nb + j] = v;
    }
  return out;
}

// Y_j = ybeta Y_j + sum_i X_i C[i * |Y| + j] (field and macro parts); with
// norms != null the weighted squared norms of the field parts of the Y_j
static void blk_comb(Ctx& c, const std::vector<BlockVec*>& X, const std::vector<BlockVec*>& Y,
                     const std::vector<double>& Cm, double ybeta, int nS, std::vector<double>* norms) {
  const int nx = (int)X.size(), ny = (int)Y.size();
  BlockVecs vx{}, vy{};
  BlockCoef cf{};
  for (int i = 0; i < nx; ++i) vx.v[i] = X[i]->a;
  for (int j = 0; j < ny; ++j) vy.v[j] = Y[j]->a;
  for (int i = 0; i < nx; ++i)
    for (int j = 0; j < ny; ++j) cf.c[i][j] = Cm[i * ny + j];
  const int nblk = pcg_block_count(c.g);
  launch_block_comb(vx, vy, nx, ny, cf, ybeta, c.g, norms ? c.blk_part : nullptr, nblk, c.st);
  for (int j = 0; j < ny; ++j)
    for (int a = 0; a < nS; ++a) {
      double v = ybeta * Y[j]->e[a];
      for (int i = 0; i < nx; ++i) v += X[i]->e[a] * Cm[i * ny + j];
      Y[j]->e[a] = v;
    }
  if (norms) {
    launch_reduce(c.blk_part, nblk, ny, c.red_dev, c.st);
    HIPCK(hipMemcpyAsync(c.red_host, c.red_dev, ny * sizeof(double), hipMemcpyDeviceToHost, c.st));
    HIPCK(hipStreamSynchronize(c.st));
    norms->assign(c.red_host, c.red_host + ny);
  }
}

// Two-level preconditioner: M(xi) everywhere except on the coarse Fourier
// set (every signed frequency |m_a| <= kc, xi != 0; one point of each
// conjugate pair on the self-conjugate planes), whose unknowns get the
// inverse of the operator's own block E there, E_ij = e_i . K e_j over the
// orthonormal coarse basis (6 per point: 3 components x real/imaginary
// unit, scaled by 1/sqrt(2), conjugate partner on the planes).
struct CoarseLevel {
  int npts = 0, m = 0;
  long long* idx = nullptr;      // device: linear half-spectrum index of every point
  long long* partner = nullptr;  // device: partner index on the planes, -1 elsewhere
  double* y = nullptr;           // device: m coordinates
  std::vector<double> L;         // Cholesky factor of E (host)
  std::vector<double> hy;
  void release() {
    for (void* p : {(void*)idx, (void*)partner, (void*)y})
      if (p) (void)hipFree(p);
    idx = partner = nullptr;
    y = nullptr;
  }
  ~CoarseLevel() { release(); }
};

static int signed_freq(int k, int n) { return k <= n / 2 ? k : k - n; }
// the wavenumber is zero on this axis (k = 0, or the Nyquist index of an even size)
static bool zero_freq(int k, int n) { return k == 0 || (n % 2 == 0 && k == n / 2); }

static void coarse_build(Ctx& c, CoarseLevel& cl, int kc, const TangentArgs<double>& tan64, void* tmp_a, void* tmp_q) {
  const Geom& g = c.g;
  std::vector<long long> hidx, hpar;
  std::vector<char> seen((size_t)g.nh, 0);
  for (int k1 = 0; k1 < g.n1; ++k1)
    for (int k2 = 0; k2 < g.n2; ++k2)
      for (int k3 = 0; k3 < g.nh3; ++k3) {
        if (std::max(std::abs(signed_freq(k1, g.n1)), std::max(std::abs(signed_freq(k2, g.n2)),
                                                              std::abs(signed_freq(k3, g.n3)))) > kc)
          continue;
        if (zero_freq(k1, g.n1) && zero_freq(k2, g.n2) && zero_freq(k3, g.n3)) continue;  // null set
        const long long k = ((long long)k1 * g.n2 + k2) * g.nh3 + k3;
        const bool plane = k3 == 0 || (g.n3 % 2 == 0 && k3 == g.n3 / 2);
        long long kp = -1;
        if (plane) {
          kp = ((long long)((g.n1 - k1) % g.n1) * g.n2 + (g.n2 - k2) % g.n2) * g.nh3 + k3;
          if (seen[kp]) continue;
          seen[k] = 1;
          if (kp == k) kp = -1;
        }
        hidx.push_back(k);
        hpar.push_back(kp);
      }
  cl.npts = (int)hidx.size();
  cl.m = 6 * cl.npts;
  if (cl.m == 0) return;
  if (cl.m > 1200) DB_THROW(DBFFT_EINVAL, "coarse_kc gives more than 1200 coarse unknowns");
  cl.idx = static_cast<long long*>(dalloc(hidx.size() * sizeof(long long)));
  cl.partner = static_cast<long long*>(dalloc(hpar.size() * sizeof(long long)));
  cl.y = static_cast<double*>(dalloc((size_t)cl.m * sizeof(double)));
  HIPCK(hipMemcpy(cl.idx, hidx.data(), hidx.size() * sizeof(long long), hipMemcpyHostToDevice));
  HIPCK(hipMemcpy(cl.partner, hpar.data(), hpar.size() * sizeof(long long), hipMemcpyHostToDevice));
  const size_t v64 = 3 * (size_t)g.nh * 2 * sizeof(double);
  std::vector<double> E((size_t)cl.m * cl.m), unit(cl.m, 0.0);
  cl.hy.assign(cl.m, 0.0);
  double zero16[16] = {0};
  HIPCK(hipMemcpyAsync(c.blk_mac, zero16, sizeof(zero16), hipMemcpyHostToDevice, c.st));
  for (int j = 0; j < cl.m; ++j) {
    // e_j, then K e_j and its coarse coordinates: column j of E
    HIPCK(hipMemsetAsync(tmp_a, 0, v64, c.st));
    unit[j] = 1.0;
    HIPCK(hipMemcpyAsync(cl.y, unit.data(), cl.m * sizeof(double), hipMemcpyHostToDevice, c.st));
    unit[j] = 0.0;
    launch_coarse_scatter(tmp_a, cl.idx, cl.partner, cl.npts, g.nh, cl.y, c.st);
    apply_K<double>(c, tmp_a, tmp_q, c.blk_mac, nullptr, tan64, c.partA, c.blk_dc, nullptr);
    launch_coarse_gather(tmp_q, cl.idx, cl.npts, g.nh, cl.y, c.st);
    HIPCK(hipMemcpyAsync(cl.hy.data(), cl.y, cl.m * sizeof(double), hipMemcpyDeviceToHost, c.st));
    HIPCK(hipStreamSynchronize(c.st));
    for (int i = 0; i < cl.m; ++i) E[(size_t)i * cl.m + j] = cl.hy[i];
  }
  for (int i = 0; i < cl.m; ++i)
    for (int j = 0; j < i; ++j) E[(size_t)i * cl.m + j] = E[(size_t)j * cl.m + i] =
                                    0.5 * (E[(size_t)i * cl.m + j] + E[(size_t)j * cl.m + i]);
  if (!chol(E, cl.m, cl.L)) DB_THROW(DBFFT_EBREAKDOWN, "coarse block of the operator not positive definite");
}

// z (= M(xi) r) gets E^-1 r on the coarse unknowns
static void coarse_apply(Ctx& c, CoarseLevel& cl, const void* r, void* z) {
  if (cl.m == 0) return;
  launch_coarse_gather(r, cl.idx, cl.npts, c.g.nh, cl.y, c.st);
  HIPCK(hipMemcpyAsync(cl.hy.data(), cl.y, cl.m * sizeof(double), hipMemcpyDeviceToHost, c.st));
  HIPCK(hipStreamSynchronize(c.st));
  cl.hy = chol_solve(cl.L, cl.m, cl.hy, 1);
  HIPCK(hipMemcpyAsync(cl.y, cl.hy.data(), cl.m * sizeof(double), hipMemcpyHostToDevice, c.st));
  launch_coarse_scatter(z, cl.idx, cl.partner, cl.npts, c.g.nh, cl.y, c.st);
}

struct BlockOut {
  int iterations = 0, applies = 0, status = DBFFT_OK;
  std::vector<int> col_iters, col_status;
};

// Solves the loads (s x 9 row-major, strain on the mask's zeros, stress on
// its ones) and fills infos[s]
static BlockOut block_solve(Ctx& c, int s, const double* loads, const int mask[9], const dbfft_opts& o,
                            dbfft_info* infos) {
  BlockOut out;
  out.col_iters.assign(s, 0);
  out.col_status.assign(s, DBFFT_ENOTCONV);
  const MacroSet ms = macro_set(c, mask);
  const int nS = ms.nS;
  double C4[81];
  mean_tangent(c, C4);
  PrecondArgs pa{};
  PcgConst pc{};
  std::memset(&pc, 0, sizeof(pc));
  build_precond(c, C4, ms, pa, pc);
  TangentArgs<double> tan64 = elastic_tangent<double>(c);
  const size_t v64 = 3 * (size_t)c.g.nh * 2 * sizeof(double);
  if (c.blk_cap < s) {
    if (c.blk) HIPCK(hipFree(c.blk));
    c.blk = nullptr;
    c.blk_cap = 0;
    c.blk = dalloc(6 * (size_t)s * v64);
    c.blk_cap = s;
  }
  if (!c.blk_mac) c.blk_mac = static_cast<double*>(dalloc(kMaxBlock * 16 * sizeof(double)));
  if (!c.blk_dc) c.blk_dc = static_cast<double*>(dalloc(kMaxBlock * 16 * sizeof(double)));
  if (!c.blk_part) c.blk_part = static_cast<double*>(dalloc((size_t)pcg_block_count(c.g) * kMaxBlock * kMaxBlock * sizeof(double)));
  std::vector<BlockVec> X(s), R(s), P(s), Q(s), Z(s), P2(s);
  {
    char* base = static_cast<char*>(c.blk);
    std::vector<BlockVec>* sets[6] = {&X, &R, &P, &Q, &Z, &P2};
    for (int k = 0; k < 6; ++k)
      for (int j = 0; j < s; ++j) (*sets[k])[j].a = base + ((size_t)k * s + j) * v64;
  }
  CoarseLevel cl;
  if (o.coarse_kc > 0) coarse_build(c, cl, o.coarse_kc, tan64, P[0].a, Q[0].a);
  // right-hand sides: R_j = -K[0; EU_j], macro rows sbar_j - B : <C : EU_j>
  std::vector<std::array<double, 9>> EU(s), sig(s);
  std::vector<std::array<double, kMaxMacro>> sbar(s);
  for (int j = 0; j < s; ++j) {
    double U_rm[9], lst[9];
    for (int i = 0; i < 9; ++i) U_rm[i] = mask[i] ? 0.0 : loads[9 * j + i];
    rm_to_stored(c.kin, U_rm, EU[j].data());
    rm_to_stored(c.kin, loads + 9 * j, lst);
    sbar[j].fill(0.0);
    for (int a = 0; a < nS; ++a) sbar[j][a] = bdot(c.kin, ms.bst[a], lst);
    set_macro(c, EU[j].data());
    apply_const<double>(c, R[j].a, c.mac_dev, tan64, c.dc_dev);
    launch_axpby<double>(R[j].a, R[j].a, 0.0, -1.0, 6 * c.g.nh, c.st);
    double d0[9];
    read_dc(c, d0);
    for (int i = 0; i < 9; ++i) sig[j][i] = d0[i];
    for (int a = 0; a < nS; ++a) R[j].e[a] = sbar[j][a] - bdot(c.kin, ms.bst[a], d0);
    HIPCK(hipMemsetAsync(X[j].a, 0, v64, c.st));
    for (int a = 0; a < kMaxMacro; ++a) X[j].e[a] = 0.0;
  }
  std::vector<double> rnorm2(s);
  {
    std::vector<BlockVec*> all;
    for (int j = 0; j < s; ++j) all.push_back(&R[j]);
    const std::vector<double> G = blk_dot(c, all, all, 0);
    for (int j = 0; j < s; ++j) rnorm2[j] = G[j * s + j];
  }
  auto converged = [&](int j, double& eq, double& ld) {
    const double nrm = frob_stored(c.kin, sig[j].data());
    const double ra = std::sqrt(std::max(rnorm2[j], 0.0));
    double rl = 0.0;
    for (int a = 0; a < nS; ++a) rl += R[j].e[a] * R[j].e[a];
    rl = std::sqrt(rl);
    eq = nrm > 0 ? ra / nrm : (ra == 0 ? 0.0 : INFINITY);
    ld = nrm > 0 ? rl / nrm : (rl == 0 ? 0.0 : INFINITY);
    return eq < o.tol && ld < o.tol_load;
  };
  std::vector<int> active;
  for (int j = 0; j < s; ++j) {
    double eq, ld;
    if (converged(j, eq, ld)) out.col_status[j] = DBFFT_OK;
    else active.push_back(j);
  }
  const int nblk = pcg_block_count(c.g);
  // Z_j = M R_j over the active columns (R_j projected onto Hermitian pairs first)
  auto precondition = [&](std::vector<BlockVec*>& Zs) {
    Zs.clear();
    for (size_t jj = 0; jj < active.size(); ++jj) {
      const int j = active[jj];
      launch_precond_init<double>(Z[j].a, R[j].a, pa, c.g, c.partB, nblk, c.st);
      coarse_apply(c, cl, R[j].a, Z[j].a);
      for (int a = 0; a < nS; ++a) {
        double v = 0.0;
        for (int b = 0; b < nS; ++b) v += pc.Me[a][b] * R[j].e[b];
        Z[j].e[a] = v;
      }
      Zs.push_back(&Z[j]);
    }
  };
  // orthonormal basis of the span of W into P2 (then swapped into P); width returned
  int m = 0;
  std::vector<BlockVec*> Pl(s), P2l(s);
  for (int j = 0; j < s; ++j) {
    Pl[j] = &P[j];
    P2l[j] = &P2[j];
  }
  // A column's pivot is the squared norm of its part orthogonal to the kept
  // columns; it is dropped as dependent when that is not above 1e-12 times
  // ref[j] (its own squared norm, or that of its preconditioned residual
  // before the conjugation).
  auto orthonormalize = [&](std::vector<BlockVec*>& W, const std::vector<double>* ref) {
    const int n = (int)W.size();
    const std::vector<double> G = blk_dot(c, W, W, nS);
    std::vector<double> d(n), Lrow(n * n, 0.0), rf(n);
    for (int i = 0; i < n; ++i) {
      d[i] = G[i * n + i];
      rf[i] = ref ? (*ref)[i] : d[i];
    }
    std::vector<int> perm, rest;
    for (int i = 0; i < n; ++i) rest.push_back(i);
    for (int t = 0; t < n; ++t) {
      std::vector<int> keep;
      for (int i : rest)
        if (d[i] > 1e-12 * rf[i]) keep.push_back(i);
      rest.swap(keep);
      if (rest.empty()) break;
      int j = rest[0];
      for (int i : rest)
        if (d[i] > d[j]) j = i;
      const double piv = std::sqrt(d[j]);
      Lrow[j * n + t] = piv;
      rest.erase(std::find(rest.begin(), rest.end(), j));
      for (int i : rest) {
        double v = G[i * n + j];
        for (int u = 0; u < t; ++u) v -= Lrow[i * n + u] * Lrow[j * n + u];
        Lrow[i * n + t] = v / piv;
        d[i] -= Lrow[i * n + t] * Lrow[i * n + t];
      }
      perm.push_back(j);
    }
    const int k = (int)perm.size();
    // C = L^-T with L the k x k factor of the kept columns (rows in pivot order)
    std::vector<double> Lk(k * k), Cm(k * k, 0.0);
    for (int t = 0; t < k; ++t)
      for (int u = 0; u < k; ++u) Lk[t * k + u] = Lrow[perm[t] * n + u];
    for (int col = 0; col < k; ++col) {
      // solve L^T c = e_col  -> column col of L^-T
      std::vector<double> e(k, 0.0);
      e[col] = 1.0;
      for (int i = k - 1; i >= 0; --i) {
        double v = e[i];
        for (int r = i + 1; r < k; ++r) v -= Lk[r * k + i] * Cm[r * k + col];
        Cm[i * k + col] = v / Lk[i * k + i];
      }
    }
    std::vector<BlockVec*> Wk(k), Yk(k);
    for (int u = 0; u < k; ++u) {
      Wk[u] = W[perm[u]];
      Yk[u] = P2l[u];
    }
    if (k > 0) blk_comb(c, Wk, Yk, Cm, 0.0, nS, nullptr);
    std::swap(Pl, P2l);
    m = k;
  };
  std::vector<BlockVec*> Zs;
  if (!active.empty()) {
    precondition(Zs);
    orthonormalize(Zs, nullptr);
  }
  while (!active.empty() && m > 0 && out.iterations < o.max_iter) {
    // Q = K P, with the mean stress of every direction
    for (int i = 0; i < m; ++i) {
      double mt[16] = {0};
      for (int a = 0; a < nS; ++a)
        for (int k = 0; k < 9; ++k) mt[k] += Pl[i]->e[a] * ms.bst[a][k];
      HIPCK(hipMemcpyAsync(c.blk_mac + 16 * i, mt, 16 * sizeof(double), hipMemcpyHostToDevice, c.st));
    }
    for (int i = 0; i < m; ++i)
      apply_K<double>(c, Pl[i]->a, Q[i].a, c.blk_mac + 16 * i, nullptr, tan64, c.partA, c.blk_dc + 16 * i, nullptr);
    double dcP[kMaxBlock][16];
    HIPCK(hipMemcpyAsync(dcP, c.blk_dc, (size_t)m * 16 * sizeof(double), hipMemcpyDeviceToHost, c.st));
    HIPCK(hipStreamSynchronize(c.st));
    out.applies += m;
    std::vector<BlockVec*> Ql(m), Ra;
    for (int i = 0; i < m; ++i) {
      Ql[i] = &Q[i];
      for (int a = 0; a < nS; ++a) Q[i].e[a] = bdot(c.kin, ms.bst[a], dcP[i]);
    }
    for (int j : active) Ra.push_back(&R[j]);
    const int na = (int)active.size();
    std::vector<BlockVec*> Pm(Pl.begin(), Pl.begin() + m);
    std::vector<double> Gam = blk_dot(c, Pm, Ql, nS);
    for (int i = 0; i < m; ++i)
      for (int k = 0; k < i; ++k) Gam[i * m + k] = Gam[k * m + i] = 0.5 * (Gam[i * m + k] + Gam[k * m + i]);
    std::vector<double> Lg;
    if (!chol(Gam, m, Lg)) {
      out.status = DBFFT_EBREAKDOWN;
      for (int j : active) out.col_status[j] = DBFFT_EBREAKDOWN;
      break;
    }
    const std::vector<double> alpha = chol_solve(Lg, m, blk_dot(c, Pm, Ra, nS), na);
    std::vector<BlockVec*> Xa;
    for (int j : active) Xa.push_back(&X[j]);
    std::vector<double> nalpha(alpha);
    for (double& v : nalpha) v = -v;
    blk_comb(c, Pm, Xa, alpha, 1.0, nS, nullptr);
    std::vector<double> rn;
    blk_comb(c, Ql, Ra, nalpha, 1.0, nS, &rn);
    for (int jj = 0; jj < na; ++jj) {
      const int j = active[jj];
      rnorm2[j] = rn[jj];
      for (int i = 0; i < m; ++i)
        for (int k = 0; k < 9; ++k) sig[j][k] += alpha[i * na + jj] * dcP[i][k];
    }
    out.iterations += 1;
    std::vector<int> still;
    for (int j : active) {
      double eq, ld;
      if (converged(j, eq, ld)) {
        out.col_status[j] = DBFFT_OK;
        out.col_iters[j] = out.iterations;
      } else {
        still.push_back(j);
      }
    }
    active.swap(still);
    if (active.empty()) break;
    precondition(Zs);
    const int nz = (int)Zs.size();
    const std::vector<double> ZZ = blk_dot(c, Zs, Zs, nS);
    std::vector<double> zref(nz);
    for (int j = 0; j < nz; ++j) zref[j] = ZZ[j * nz + j];
    const std::vector<double> beta0 = chol_solve(Lg, m, blk_dot(c, Ql, Zs, nS), nz);
    std::vector<double> beta(beta0);
    for (double& v : beta) v = -v;
    blk_comb(c, Pm, Zs, beta, 1.0, nS, nullptr);
    orthonormalize(Zs, &zref);
  }
  for (int j : active) out.col_iters[j] = out.iterations;
  // true residuals and averages of every column
  for (int j = 0; j < s; ++j) {
    double mt[9], sig_st[9], eq, ld;
    for (int i = 0; i < 9; ++i) {
      mt[i] = EU[j][i];
      for (int a = 0; a < nS; ++a) mt[i] += X[j].e[a] * ms.bst[a][i];
    }
    evaluate_linear(c, static_cast<const double*>(X[j].a), mt, ms, sbar[j].data(), sig_st, eq, ld);
    dbfft_info& inf = infos[j];
    std::memset(&inf, 0, sizeof(inf));
    inf.pcg_iters = out.col_iters[j];
    inf.increments = 1;
    inf.status = out.col_status[j];
    inf.eq_res = eq;
    inf.load_res = ld;
    stored_to_rm(c.kin, sig_st, inf.sigma_bar);
    stored_to_rm(c.kin, mt, inf.eps_bar);
    if (out.col_status[j] != DBFFT_OK && out.status == DBFFT_OK) out.status = out.col_status[j];
  }
  return out;
}

// ------------------------------------------------------------------ Newton
static void material_update(Ctx& c, const double* fld, double* sig_out, double dt) {
  HIPCK(hipMemsetAsync(c.fail_dev, 0, sizeof(int), c.st));
  if (c.mat == DBFFT_MAT_J2VP_CUBIC) {
    launch_j2_update(fld, c.state, c.grain, c.grainC, c.grainS, c.j2_s0, c.j2_m, c.j2_edot0, dt, c.g.nvox, sig_out,
                     c.tanf, c.state_new, c.fail_dev, c.st);
  } else {
    NeoParams np;
    for (int i = 0; i < kMaxPhases; ++i) {
      np.mu[i] = c.mu[i];
      np.lam[i] = c.lam[i];
    }
    if (c.mat == DBFFT_MAT_SVK) launch_svk_update(fld, c.phase, np, c.g.nvox, sig_out, c.tanf, c.fail_dev, c.st);
    else launch_neo_update(fld, c.phase, np, c.g.nvox, sig_out, c.tanf, c.fail_dev, c.st);
  }
  int fail = 0;
  HIPCK(hipMemcpyAsync(&fail, c.fail_dev, sizeof(int), hipMemcpyDeviceToHost, c.st));
  HIPCK(hipStreamSynchronize(c.st));
  if (fail) DB_THROW(DBFFT_EMATERIAL, "constitutive update failed (local Newton or J <= 0)");
  c.tangent_from_field = 1;
  if (c.prec == DBFFT_FP32_MIXED) {
    const int nt = (c.mat == DBFFT_MAT_J2VP_CUBIC) ? 21 : (c.mat == DBFFT_MAT_SVK ? 15 : 10);
    launch_convert<double, float>(c.tanf32, c.tanf, (long long)nt * c.g.nvox, c.st);
  }
}

static double max_abs_diff(Ctx& c, const double* a, const double* b, long long n) {
  const int nb = 512;
  launch_max_abs_diff(a, b, n, c.partA, nb, c.st);
  std::vector<double> h(nb);
  HIPCK(hipMemcpyAsync(h.data(), c.partA, nb * sizeof(double), hipMemcpyDeviceToHost, c.st));
  HIPCK(hipStreamSynchronize(c.st));
  double m = 0.0;
  for (double v : h) m = std::max(m, v);
  return m;
}

// Newton state of one cell (Sec. 2.4): the increments of the load path, the
// macro unknown e on the stress-controlled set, the preconditioner of the
// current mean tangent and the bookkeeping of the current increment.
struct NewtonState {
  MacroSet ms;
  int mask[9];
  double load_rm[9];
  int ninc = 1;
  double dt = 1.0;
  dbfft_opts o;
  double e[kMaxMacro] = {0};
  double EU[9] = {0};
  double sbar[kMaxMacro] = {0};
  double sig_st[9] = {0};
  double re[kMaxMacro] = {0};
  PrecondArgs pa;
  PcgConst pc;
  bool have_pre = false;
  int status = DBFFT_OK;
  int k = 0, i = 0;
  double dmax = INFINITY;
  bool conv = false;
  dbfft_info info;
};

// doubles per increment in the checkpoint buffer
static size_t ck_stride(const Ctx& c) { return 6 * (size_t)c.g.nh + 6 * (size_t)c.g.nvox; }

static void macro_total(const Ctx& c, const NewtonState& S, double mt[9]) {
  for (int i = 0; i < 9; ++i) mt[i] = S.EU[i];
  for (int a = 0; a < S.ms.nS; ++a)
    for (int i = 0; i < 9; ++i) mt[i] += S.e[a] * S.ms.bst[a][i];
  (void)c;
}

static void newton_init(Ctx& c, NewtonState& S, const double load_rm[9], const int mask[9], int ninc, double dt,
                        const dbfft_opts& o) {
  S.ms = macro_set(c, mask);
  for (int i = 0; i < 9; ++i) {
    S.mask[i] = mask[i];
    S.load_rm[i] = load_rm[i];
  }
  S.ninc = ninc;
  S.dt = dt;
  S.o = o;
  std::memset(&S.pc, 0, sizeof(S.pc));
  std::memset(&S.info, 0, sizeof(S.info));
  HIPCK(hipMemsetAsync(c.sol, 0, 3 * (size_t)c.g.nh * 2 * sizeof(double), c.st));
  if (c.mat == DBFFT_MAT_J2VP_CUBIC) HIPCK(hipMemsetAsync(c.state, 0, 6 * c.g.nvox * sizeof(double), c.st));
  c.ck_n = 0;
  if (c.mat == DBFFT_MAT_J2VP_CUBIC && o.checkpoint) {
    if (c.ck_cap < ninc) {
      HIPCK(hipStreamSynchronize(c.st));
      if (c.ck_buf) HIPCK(hipFree(c.ck_buf));
      c.ck_buf = nullptr;
      c.ck_cap = 0;
      c.ck_buf = static_cast<double*>(dalloc((size_t)ninc * ck_stride(c) * sizeof(double)));
      c.ck_cap = ninc;
    }
    c.ck_mt.assign(ninc, std::array<double, 9>{});
    c.ck_dt = dt;
  }
}

// prescribed parts of increment k, strain field of the current iterate
static void newton_begin_increment(Ctx& c, NewtonState& S, int k) {
  S.k = k;
  S.i = 0;
  S.dmax = INFINITY;
  S.conv = false;
  const double frac = (double)k / (double)S.ninc;
  double lrm[9], U_rm[9];
  for (int i = 0; i < 9; ++i) {
    double v = S.load_rm[i];
    if (c.kin == KIN_FINITE && !S.mask[i] && (i % 4 == 0)) v -= 1.0;  // F - I
    lrm[i] = frac * v;
    U_rm[i] = S.mask[i] ? 0.0 : lrm[i];
  }
  rm_to_stored(c.kin, U_rm, S.EU);
  double lst[9];
  rm_to_stored(c.kin, lrm, lst);
  for (int a = 0; a < S.ms.nS; ++a) S.sbar[a] = bdot(c.kin, S.ms.bst[a], lst);
  double mt[9];
  macro_total(c, S, mt);
  set_macro(c, mt);
  strain_field(c, c.sol, c.mac_dev, c.fa);
}

// constitutive update, preconditioner refresh and residual at the current
// iterate.  Returns 1 when the Newton test passes, 0 when a linear
// correction is needed, -1 when the Newton cap is reached.
static int newton_evaluate(Ctx& c, NewtonState& S) {
  material_update(c, c.fa, c.fc, S.dt);
  if (!S.have_pre || (S.i == 0 && S.o.refresh == 0)) {
    double C4[81];
    mean_tangent(c, C4);
    build_precond(c, C4, S.ms, S.pa, S.pc);
    S.have_pre = true;
  }
  stress_residual(c, c.fc, c.t64, c.dc_dev);
  read_dc(c, S.sig_st);
  for (int a = 0; a < kMaxMacro; ++a) S.re[a] = 0.0;
  for (int a = 0; a < S.ms.nS; ++a) S.re[a] = S.sbar[a] - bdot(c.kin, S.ms.bst[a], S.sig_st);
  if (g_verbose) {
    double rl = 0.0;
    for (int a = 0; a < S.ms.nS; ++a) rl += S.re[a] * S.re[a];
    std::fprintf(stderr, "[dbfft] newton inc %d it %d dmax %.3e |r_e| %.3e sig0 %.4e\n", S.k, S.i, S.dmax,
                 std::sqrt(rl), S.sig_st[0]);
  }
  if (S.i > 0 && S.dmax < S.o.newton_tol) {
    S.conv = true;
    return 1;
  }
  if (S.i >= S.o.max_newton) return -1;
  S.pc.tol = S.o.tol;
  S.pc.tol_load = S.o.tol_load;
  S.pc.max_iter = S.o.max_iter;
  // right-hand side of the linear correction in the PCG precision
  if (c.prec == DBFFT_FP64)
    HIPCK(hipMemcpyAsync(c.r, c.t64, 3 * (size_t)c.g.nh * 2 * sizeof(double), hipMemcpyDeviceToDevice, c.st));
  else
    launch_convert<double, float>(c.r, c.t64, 6 * c.g.nh, c.st);
  return 0;
}

// adds the PCG correction (in c.x) and re-evaluates the strain field
static void newton_apply_correction(Ctx& c, NewtonState& S, const PcgOut& po) {
  S.info.pcg_iters += po.iters;
  S.info.newton_iters += 1;
  if (po.status == 2) {
    S.status = DBFFT_EBREAKDOWN;
    return;
  }
  if (po.status == 3) {
    S.status = DBFFT_ENOTCONV;
    return;
  }
  if (c.prec == DBFFT_FP64) {
    launch_axpby<double>(c.sol, c.x, 1.0, 1.0, 6 * c.g.nh, c.st);
  } else {
    launch_convert<float, double>(c.q, c.x, 6 * c.g.nh, c.st);
    launch_axpby<double>(c.sol, c.q, 1.0, 1.0, 6 * c.g.nh, c.st);
  }
  for (int a = 0; a < S.ms.nS; ++a) S.e[a] += po.xe[a];
  double mt[9];
  macro_total(c, S, mt);
  set_macro(c, mt);
  std::swap(c.fa, c.fb);
  strain_field(c, c.sol, c.mac_dev, c.fa);
  S.dmax = max_abs_diff(c, c.fa, c.fb, (long long)c.ncomp * c.g.nvox);
  S.i += 1;
}

static void newton_end_increment(Ctx& c, NewtonState& S) {
  if (c.mat == DBFFT_MAT_J2VP_CUBIC && S.o.checkpoint) {
    double* ck = c.ck_buf + (size_t)(S.k - 1) * ck_stride(c);
    HIPCK(hipMemcpyAsync(ck, c.sol, 6 * (size_t)c.g.nh * sizeof(double), hipMemcpyDeviceToDevice, c.st));
    HIPCK(hipMemcpyAsync(ck + 6 * (size_t)c.g.nh, c.state, 6 * (size_t)c.g.nvox * sizeof(double),
                         hipMemcpyDeviceToDevice, c.st));
    macro_total(c, S, c.ck_mt[S.k - 1].data());
    c.ck_n = S.k;
  }
  if (c.mat == DBFFT_MAT_J2VP_CUBIC) std::swap(c.state, c.state_new);
  S.info.increments += 1;
}

// residuals and averages of the final state into the context and info
static void newton_finish(Ctx& c, NewtonState& S) {
  const double ra = std::sqrt(std::max(dot64(c, c.t64, c.t64), 0.0));
  const double nrm = frob_stored(c.kin, S.sig_st);
  S.info.eq_res = nrm > 0 ? ra / nrm : 0.0;
  double rl = 0.0;
  {
    double lrm[9], lst[9];
    const double frac = (double)std::max(S.info.increments, 1) / (double)S.ninc;
    for (int i = 0; i < 9; ++i) lrm[i] = frac * S.load_rm[i];
    rm_to_stored(c.kin, lrm, lst);
    for (int a = 0; a < S.ms.nS; ++a) {
      const double d = bdot(c.kin, S.ms.bst[a], lst) - bdot(c.kin, S.ms.bst[a], S.sig_st);
      rl += d * d;
    }
  }
  S.info.load_res = nrm > 0 ? std::sqrt(rl) / nrm : 0.0;
  double et[9] = {0};
  for (int a = 0; a < S.ms.nS; ++a)
    for (int i = 0; i < 9; ++i) et[i] += S.e[a] * S.ms.bst[a][i];
  for (int i = 0; i < 9; ++i) c.e_st[i] = et[i];
  for (int i = 0; i < 9; ++i) c.EU_st[i] = S.EU[i];
  double avg_st[9];
  for (int i = 0; i < 9; ++i) avg_st[i] = S.EU[i] + et[i];
  stored_to_rm(c.kin, S.sig_st, c.sig_rm);
  stored_to_rm(c.kin, avg_st, c.eps_rm);
  if (c.kin == KIN_FINITE)
    for (int i = 0; i < 9; i += 4) c.eps_rm[i] += 1.0;  // <F> = I + <H>
  for (int i = 0; i < 9; ++i) {
    S.info.sigma_bar[i] = c.sig_rm[i];
    S.info.eps_bar[i] = c.eps_rm[i];
  }
  S.info.status = S.status;
}

static int newton_solve(Ctx& c, const double load_rm[9], const int mask[9], int ninc, double dt,
                        const dbfft_opts& o, dbfft_info& info) {
  NewtonState S;
  newton_init(c, S, load_rm, mask, ninc, dt, o);
  for (int k = 1; k <= ninc && S.status == DBFFT_OK; ++k) {
    newton_begin_increment(c, S, k);
    for (;;) {
      const int ev = newton_evaluate(c, S);
      if (ev == 1) break;
      if (ev < 0) {
        S.status = DBFFT_ENOTCONV;
        break;
      }
      PcgOut po;
      if (c.prec == DBFFT_FP64) {
        TangentArgs<double> tan = elastic_tangent<double>(c);
        po = run_pcg<double>(c, tan, S.pa, S.pc, c.x, c.r, c.p, c.q, S.sig_st, S.re, o.check_every);
      } else {
        TangentArgs<float> tan = elastic_tangent<float>(c);
        po = run_pcg<float>(c, tan, S.pa, S.pc, c.x, c.r, c.p, c.q, S.sig_st, S.re, o.check_every);
      }
      newton_apply_correction(c, S, po);
      if (S.status != DBFFT_OK) break;
    }
    if (S.status != DBFFT_OK) break;
    newton_end_increment(c, S);
  }
  newton_finish(c, S);
  info = S.info;
  return S.status;
}

// ------------------------------------------------------------------ setup
static bool smooth(long long n) {
  if (n < 1) return false;
  for (int p : {2, 3, 5, 7})
    while (n % p == 0) n /= p;
  return n == 1;
}

static void release(Ctx* c) {
  for (dbfft_ctx* h : c->helpers) dbfft_destroy(h);
  for (hipStream_t s : c->helper_streams) (void)hipStreamDestroy(s);
  c->helpers.clear();
  c->helper_streams.clear();
  (void)hipStreamSynchronize(c->st);
  void* dev[] = {c->td.tw1, c->td.tw2, c->td.tw3, c->td.rtw, c->tf.tw1, c->tf.tw2, c->tf.tw3, c->tf.rtw,
                 c->phase, c->E64, c->E32, c->grain, c->grain21, c->grainC, c->grainS, c->W, c->x, c->r, c->p,
                 c->q, c->b, c->t64, c->sol, c->sol2, c->fa, c->fb, c->fc, c->state, c->state_new, c->tanf,
                 c->tanf32, c->partA, c->partB, c->sc_dev, c->dc_dev, c->mac_dev, c->red_dev, c->fail_dev,
                 c->ck_buf, c->adj_lam, c->blk, c->blk_mac, c->blk_dc, c->blk_part};
  for (void* p : dev)
    if (p) (void)hipFree(p);
  if (c->sc_host) (void)hipHostFree(c->sc_host);
  if (c->red_host) (void)hipHostFree(c->red_host);
  for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
  for (hipEvent_t e : c->ext_pool) (void)hipEventDestroy(e);
  if (c->chunk_exec) (void)hipGraphExecDestroy(c->chunk_exec);
  if (c->chunk_graph) (void)hipGraphDestroy(c->chunk_graph);
  if (c->cap_st) (void)hipStreamDestroy(c->cap_st);
}

// grid checks shared by every entry point that takes a grid: smooth sizes,
// and the LDS limits of the x/y passes (one line plus twiddles per tile
// column) and of the z pass (one z line of every component), 64 KiB each
static void check_grid(const int64_t n[3], int kin) {
  if (!n) DB_THROW(DBFFT_EINVAL, "null grid size");
  for (int a = 0; a < 3; ++a)
    if (n[a] < 1 || n[a] > 4096 || !smooth(n[a])) DB_THROW(DBFFT_EINVAL, "grid sizes must be 2^a 3^b 5^c 7^d");
  const int nc = (kin == DBFFT_FINITE) ? 9 : 6;
  for (int a = 0; a < 2; ++a)
    if ((size_t)3 * n[a] * 16 > 64 * 1024) DB_THROW(DBFFT_EUNSUPPORTED, "n1 and n2 must be <= 1365");
  const size_t M = (size_t)n[2] / 2;
  if ((2 * M + 1) * 16 + 2 * M * 16 + (M + 1) * 16 + (size_t)nc * n[2] * 8 > 64 * 1024)
    DB_THROW(DBFFT_EUNSUPPORTED, "n3 too large for the z pass");
}

// geometry and transform plans of a checked grid (host only, allocates nothing)
static void init_grid(Ctx* c, const int64_t n[3], int kin, int prec, int mat, void* stream) {
  for (int a = 0; a < 3; ++a) c->n[a] = (int)n[a];
  c->kin = kin;
  c->prec = prec;
  c->mat = mat;
  c->ncomp = (kin == DBFFT_SMALL) ? 6 : 9;
  c->st = static_cast<hipStream_t>(stream);
  Geom& g = c->g;
  g.n1 = c->n[0];
  g.n2 = c->n[1];
  g.n3 = c->n[2];
  g.nh3 = g.n3 / 2 + 1;
  g.nh = (long long)g.n1 * g.n2 * g.nh3;
  g.nvox = (long long)g.n1 * g.n2 * g.n3;
  g.inv_nvox = 1.0 / (double)g.nvox;
  g.il1 = g.il2 = g.il3 = 1.0;
  if (!make_plan(g.n1, c->p1) || !make_plan(g.n2, c->p2) || !make_plan(z_length(g.n3), c->p3))
    DB_THROW(DBFFT_EINVAL, "cannot plan the transform lengths");
}

// partial sums any kernel of a context writes (energy, CG dots, mean tangent)
static int partial_count(const Geom& g) {
  const int zparts = std::max(std::max(mixed_line_supported(g.n3, 16, true) ? mixed_line_energy_blocks(g, true) : 0,
                                       odd_line_supported(g.n3) ? odd_line_energy_blocks(g) : 0),
                              staged_line_supported(g.n3, 8, false, false) ? staged_line_blocks(g) : 0);
  return std::max(std::max(std::max(std::max(line_block_count(g), 2 * pcg_block_count(g)),
                                    tangent_mean_block_count(g) * 81),
                           fused_cg_partials(g)),
                  zparts) + 64;
}

// Lame constants of the (E, nu) pairs of an isotropic phase table
static void iso_phase_table(const double* params, int nparams, int& nphase, double* lam, double* mu) {
  if (nparams % 2 != 0 || nparams / 2 > kMaxPhases) DB_THROW(DBFFT_EINVAL, "phase parameters: pairs, at most 8 phases");
  nphase = nparams / 2;
  for (int p = 0; p < nphase; ++p) {
    const double a = params[2 * p], b = params[2 * p + 1];
    lam[p] = a * b / ((1.0 + b) * (1.0 - 2.0 * b));
    mu[p] = a / (2.0 * (1.0 + b));
  }
}

static void setup(Ctx* c, const int64_t n[3], int kin, int prec, int mat, const void* field, const double* params,
                  int nparams, void* stream) {
  check_grid(n, kin);
  if (kin != DBFFT_SMALL && kin != DBFFT_FINITE) DB_THROW(DBFFT_EINVAL, "unknown kinematics");
  if (prec != DBFFT_FP64 && prec != DBFFT_FP32_MIXED) DB_THROW(DBFFT_EINVAL, "unknown precision");
  if (mat < 0 || mat > DBFFT_MAT_SVK) DB_THROW(DBFFT_EINVAL, "unknown material kind");
  if ((mat == DBFFT_MAT_NEOHOOKE || mat == DBFFT_MAT_SVK) != (kin == DBFFT_FINITE))
    DB_THROW(DBFFT_EINVAL, "NEOHOOKE and SVK need FINITE kinematics and every other material SMALL");
  if (!field) DB_THROW(DBFFT_EINVAL, "null material field");
  if (!params || nparams < 1) DB_THROW(DBFFT_EINVAL, "null material parameters");
  c->setup_params.assign(params, params + nparams);
  HIPCK(hipGetDevice(&c->dev));

  {
    init_grid(c, n, kin, prec, mat, stream);
    Geom& g = c->g;
    std::vector<double> re, im;
    twiddles(g.n1, g.n1, g.n1, re, im);
    c->td.tw1 = upload_table<double>(re, im);
    c->tf.tw1 = upload_table<float>(re, im);
    twiddles(g.n2, g.n2, g.n2, re, im);
    c->td.tw2 = upload_table<double>(re, im);
    c->tf.tw2 = upload_table<float>(re, im);
    const int M = g.n3 / 2, Z = z_length(g.n3);
    twiddles(Z, Z, std::max(Z, 1), re, im);
    c->td.tw3 = upload_table<double>(re, im);
    c->tf.tw3 = upload_table<float>(re, im);
    twiddles(g.n3, g.n3, M + 1, re, im);
    c->td.rtw = upload_table<double>(re, im);
    c->tf.rtw = upload_table<float>(re, im);

    const long long N = g.nvox;
    // material
    if (mat == DBFFT_MAT_ISO_PHASE || mat == DBFFT_MAT_NEOHOOKE || mat == DBFFT_MAT_SVK) {
      iso_phase_table(params, nparams, c->nphase, c->lam, c->mu);
      if (mat == DBFFT_MAT_NEOHOOKE)
        for (int p = 0; p < c->nphase; ++p) {
          // (mu, kappa) pairs: lambda = kappa - 2 mu / 3
          c->mu[p] = params[2 * p];
          c->lam[p] = params[2 * p + 1] - 2.0 * params[2 * p] / 3.0;
        }
      std::vector<uint8_t> hp(N);
      HIPCK(hipMemcpy(hp.data(), field, N, hipMemcpyDeviceToHost));
      for (long long v = 0; v < N; ++v)
        if (hp[v] >= c->nphase) DB_THROW(DBFFT_EINVAL, "phase id out of range");
      c->phase = static_cast<uint8_t*>(dalloc(N));
      HIPCK(hipMemcpy(c->phase, field, N, hipMemcpyDeviceToDevice));
    } else if (mat == DBFFT_MAT_ISO_FIELD) {
      c->nu = params[0];
      c->lam1 = c->nu / ((1.0 + c->nu) * (1.0 - 2.0 * c->nu));
      c->mu1 = 1.0 / (2.0 * (1.0 + c->nu));
      c->E64 = static_cast<double*>(dalloc(N * sizeof(double)));
      HIPCK(hipMemcpy(c->E64, field, N * sizeof(double), hipMemcpyDeviceToDevice));
      c->E32 = static_cast<float*>(dalloc(N * sizeof(float)));
      launch_convert<double, float>(c->E32, c->E64, N, c->st);
    } else {
      // grain based
      std::vector<int32_t> hg(N);
      HIPCK(hipMemcpy(hg.data(), field, N * sizeof(int32_t), hipMemcpyDeviceToHost));
      int gmax = -1;
      for (long long v = 0; v < N; ++v) {
        if (hg[v] < 0) DB_THROW(DBFFT_EINVAL, "negative grain id");
        gmax = std::max(gmax, (int)hg[v]);
      }
      std::vector<double> C36;
      if (mat == DBFFT_MAT_ANISO_GRAIN) {
        c->ngrain = nparams / 36;
        if (c->ngrain * 36 != nparams || c->ngrain <= gmax) DB_THROW(DBFFT_EINVAL, "ANISO_GRAIN needs 36 values per grain id");
        C36.assign(params, params + nparams);
      } else {
        if (nparams < 6 || (nparams - 6) % 9 != 0) DB_THROW(DBFFT_EINVAL, "J2VP_CUBIC parameters: 6 + 9 per grain");
        c->ngrain = (nparams - 6) / 9;
        if (c->ngrain <= gmax) DB_THROW(DBFFT_EINVAL, "grain id without rotation");
        const double c11 = params[0], c12 = params[1], c44 = params[2];
        c->j2_s0 = params[3];
        c->j2_m = params[4];
        c->j2_edot0 = params[5];
        double Cc[81] = {0};
        for (int i = 0; i < 3; ++i)
          for (int j = 0; j < 3; ++j) {
            if (i == j) Cc[((i * 3 + i) * 3 + i) * 3 + i] = c11;
            else {
              Cc[((i * 3 + i) * 3 + j) * 3 + j] = c12;
              Cc[((i * 3 + j) * 3 + i) * 3 + j] = c44;
              Cc[((i * 3 + j) * 3 + j) * 3 + i] = c44;
            }
          }
        C36.assign((size_t)c->ngrain * 36, 0.0);
        double B[6][9];
        for (int a = 0; a < 6; ++a) mandel_tensor(a, B[a]);
        for (int gi = 0; gi < c->ngrain; ++gi) {
          const double* R = params + 6 + 9 * gi;
          // C'_ijkl = R_ia R_jb R_kc R_ld C_abcd, then Mandel B_a : C' : B_b
          std::vector<double> Cr(81, 0.0);
          for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j)
              for (int k = 0; k < 3; ++k)
                for (int l = 0; l < 3; ++l) {
                  double s = 0.0;
                  for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b)
                      for (int cc = 0; cc < 3; ++cc)
                        for (int d = 0; d < 3; ++d) {
                          const double cv = Cc[((a * 3 + b) * 3 + cc) * 3 + d];
                          if (cv != 0.0) s += R[i * 3 + a] * R[j * 3 + b] * R[k * 3 + cc] * R[l * 3 + d] * cv;
                        }
                  Cr[((i * 3 + j) * 3 + k) * 3 + l] = s;
                }
          for (int a = 0; a < 6; ++a)
            for (int b = 0; b < 6; ++b) {
              double s = 0.0;
              for (int ij = 0; ij < 9; ++ij)
                for (int kl = 0; kl < 9; ++kl) s += B[a][ij] * Cr[ij * 9 + kl] * B[b][kl];
              C36[(size_t)gi * 36 + a * 6 + b] = s;
            }
        }
      }
      std::vector<double> t21((size_t)c->ngrain * 21), S36((size_t)c->ngrain * 36);
      for (int gi = 0; gi < c->ngrain; ++gi) {
        int idx = 0;
        for (int a = 0; a < 6; ++a)
          for (int b = a; b < 6; ++b)
            t21[(size_t)gi * 21 + idx++] = 0.5 * (C36[(size_t)gi * 36 + a * 6 + b] + C36[(size_t)gi * 36 + b * 6 + a]);
        std::vector<double> A(C36.begin() + (size_t)gi * 36, C36.begin() + (size_t)gi * 36 + 36), X;
        if (!small_inverse(A, 6, X)) DB_THROW(DBFFT_EINVAL, "singular grain stiffness");
        for (int i = 0; i < 36; ++i) S36[(size_t)gi * 36 + i] = X[i];
      }
      c->grain = static_cast<int32_t*>(dalloc(N * sizeof(int32_t)));
      HIPCK(hipMemcpy(c->grain, field, N * sizeof(int32_t), hipMemcpyDeviceToDevice));
      c->grain21 = static_cast<double*>(dalloc(t21.size() * sizeof(double)));
      HIPCK(hipMemcpy(c->grain21, t21.data(), t21.size() * sizeof(double), hipMemcpyHostToDevice));
      c->grainC = static_cast<double*>(dalloc(C36.size() * sizeof(double)));
      HIPCK(hipMemcpy(c->grainC, C36.data(), C36.size() * sizeof(double), hipMemcpyHostToDevice));
      c->grainS = static_cast<double*>(dalloc(S36.size() * sizeof(double)));
      HIPCK(hipMemcpy(c->grainS, S36.data(), S36.size() * sizeof(double), hipMemcpyHostToDevice));
    }

    // workspaces
    const size_t vb = 3 * (size_t)g.nh * 2 * sizeof(double);
    c->W = dalloc((size_t)c->ncomp * g.nh * 2 * sizeof(double));
    c->x = dalloc(vb);
    c->r = dalloc(vb);
    c->p = dalloc(vb);
    c->q = dalloc(vb);
    c->b = dalloc(vb);
    c->t64 = dalloc(vb);
    c->sol = static_cast<double*>(dalloc(vb));
    HIPCK(hipMemset(c->sol, 0, vb));
    const size_t fbytes = (size_t)c->ncomp * N * sizeof(double);
    c->fa = static_cast<double*>(dalloc(fbytes));
    c->fb = static_cast<double*>(dalloc(fbytes));
    c->fc = static_cast<double*>(dalloc(fbytes));
    if (mat == DBFFT_MAT_J2VP_CUBIC) {
      c->state = static_cast<double*>(dalloc(6 * N * sizeof(double)));
      c->state_new = static_cast<double*>(dalloc(6 * N * sizeof(double)));
      HIPCK(hipMemset(c->state, 0, 6 * N * sizeof(double)));
      c->tanf = static_cast<double*>(dalloc(21 * N * sizeof(double)));
      c->tanf32 = static_cast<float*>(dalloc(21 * N * sizeof(float)));
    } else if (mat == DBFFT_MAT_SVK) {
      c->tanf = static_cast<double*>(dalloc(15 * N * sizeof(double)));
      c->tanf32 = static_cast<float*>(dalloc(15 * N * sizeof(float)));
      // reference configuration: F = I, S = 0
      std::vector<double> h(15 * N, 0.0);
      for (long long v = 0; v < N; ++v) h[0 * N + v] = h[4 * N + v] = h[8 * N + v] = 1.0;
      HIPCK(hipMemcpy(c->tanf, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice));
      launch_convert<double, float>(c->tanf32, c->tanf, 15 * N, c->st);
    } else if (mat == DBFFT_MAT_NEOHOOKE) {
      c->tanf = static_cast<double*>(dalloc(10 * N * sizeof(double)));
      c->tanf32 = static_cast<float*>(dalloc(10 * N * sizeof(float)));
      // reference configuration: F^-1 = I, ln J = 0
      std::vector<double> h(10 * N, 0.0);
      for (long long v = 0; v < N; ++v) h[0 * N + v] = h[4 * N + v] = h[8 * N + v] = 1.0;
      HIPCK(hipMemcpy(c->tanf, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice));
      launch_convert<double, float>(c->tanf32, c->tanf, 10 * N, c->st);
    }
    const int nparts = partial_count(g);
    c->npart = nparts;
    c->partA = static_cast<double*>(dalloc(nparts * sizeof(double)));
    c->partB = static_cast<double*>(dalloc(nparts * sizeof(double)));
    c->sc_dev = static_cast<PcgScalars*>(dalloc(sizeof(PcgScalars)));
    HIPCK(hipHostMalloc((void**)&c->sc_host, sizeof(PcgScalars), hipHostMallocDefault));
    c->dc_dev = static_cast<double*>(dalloc(16 * sizeof(double)));
    HIPCK(hipMemset(c->dc_dev, 0, 16 * sizeof(double)));
    c->mac_dev = static_cast<double*>(dalloc(16 * sizeof(double)));
    HIPCK(hipMemset(c->mac_dev, 0, 16 * sizeof(double)));
    c->red_dev = static_cast<double*>(dalloc(128 * sizeof(double)));
    HIPCK(hipHostMalloc((void**)&c->red_host, 128 * sizeof(double), hipHostMallocDefault));
    c->fail_dev = static_cast<int*>(dalloc(sizeof(int)));
    HIPCK(hipStreamSynchronize(c->st));
  }
}

// ------------------------------------------------------------------ batches
// A batch groups contexts of one precision and kinematics (any grid sizes).
// Every batched PCG iteration is one launch per pass over all cells; a
// chunk of iterations is captured once in a HIP graph and replayed.
struct Batch {
  std::vector<Ctx*> cells;
  std::vector<dbfft_ctx*> handles;  // the callers' handles of `cells`
  int prec = 0, kin = 0, ncomp = 6;
  hipStream_t st = nullptr;  // own stream (graph capture needs a non-null stream)
  void* desc_dev = nullptr;
  size_t desc_size = 0;
  std::vector<unsigned char> desc_host;
  int* boff_dev = nullptr;
  BatchLaunch bl;
  int* flags_dev = nullptr;
  int* flags_host = nullptr;
  bool use_graph = true;
  int chunk = 8, graph_chunk = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<int> tzx, tzy, L, mx, my, mz;
  std::vector<hipStream_t> lane_st;  // streams of the cell-by-cell lanes (created on first use)
};

template <typename T>
static void fill_desc(Batch& B, int r, CellDesc<T>& D) {
  Ctx& c = *B.cells[r];
  Tables<T>& tb = tables<T>(c);
  D.g = c.g;
  D.p1 = c.p1;
  D.p2 = c.p2;
  D.p3 = c.p3;
  D.tw1 = static_cast<const cpx<T>*>(tb.tw1);
  D.tw2 = static_cast<const cpx<T>*>(tb.tw2);
  D.tw3 = static_cast<const cpx<T>*>(tb.tw3);
  D.rtw = static_cast<const cpx<T>*>(tb.rtw);
  D.W = static_cast<cpx<T>*>(c.W);
  D.x = static_cast<cpx<T>*>(c.x);
  D.r = static_cast<cpx<T>*>(c.r);
  D.p = static_cast<cpx<T>*>(c.p);
  D.q = static_cast<cpx<T>*>(c.q);
  D.tan = elastic_tangent<T>(c);
  D.sc = c.sc_dev;
  D.partA = c.partA;
  D.partB = c.partB;
  D.dc = c.dc_dev;
  D.tzx = B.tzx[r];
  D.tzy = B.tzy[r];
  D.L = B.L[r];
  D.mx = B.mx[r];
  D.my = B.my[r];
  D.mz = B.mz[r];
}

// two-step shapes (the host side of MixedShape / MixedLine)
static int two_step_threads(int n) {
  const int n1 = mixed_n1(n), n2 = n / n1;
  return n1 > n2 ? n1 : n2;
}
static int two_step_tz(int n) {
  const int tl = two_step_threads(n);
  return (256 / tl) < 32 ? (256 / tl) : 32;
}

template <typename T>
static void batch_build(Batch& B) {
  const int n = (int)B.cells.size();
  B.desc_size = sizeof(CellDesc<T>);
  B.desc_host.assign(B.desc_size * n, 0);
  const int eb = (int)(2 * sizeof(T));
  B.tzx.assign(n, 8);
  B.tzy.assign(n, 8);
  B.L.assign(n, 1);
  B.mx.assign(n, 0);
  B.my.assign(n, 0);
  B.mz.assign(n, 0);
  for (int r = 0; r < n; ++r) {
    Ctx& c = *B.cells[r];
    B.mx[r] = batch_two_step_xy(c.n[0]) ? 1 : 0;
    B.my[r] = batch_two_step_xy(c.n[1]) ? 1 : 0;
    const int kind = elastic_tangent<T>(c).kind;
    const bool iso = c.kin == KIN_SMALL && (kind == TAN_ISO_PHASE || kind == TAN_ISO_FIELD);
    if (batch_two_step_z(c.n[2] / 2) && c.n[2] % 2 == 0) B.mz[r] = iso ? 1 : (sizeof(T) == 4 ? 2 : 0);
    if (B.mx[r]) B.tzx[r] = two_step_tz(c.n[0]);
    if (B.my[r]) B.tzy[r] = two_step_tz(c.n[1]);
  }
  std::vector<int> bx(n + 1, 0), by(n + 1, 0), bz(n + 1, 0), bv(n + 1, 0);
  size_t lx = 0, ly = 0, lz = 0;
  for (int r = 0; r < n; ++r) {
    Ctx& c = *B.cells[r];
    B.L[r] = line_lines_per_block(c.g, c.ncomp, eb);
  }
  // tile autotuner: time one plain pass per candidate column-tile width
  for (int r = 0; r < n; ++r) {
    Ctx& c = *B.cells[r];
    int reuse = -1;
    for (int q = 0; q < r; ++q)
      if (B.cells[q]->n[0] == c.n[0] && B.cells[q]->n[1] == c.n[1] && B.cells[q]->n[2] == c.n[2]) reuse = q;
    if (reuse >= 0) {
      B.tzx[r] = B.tzx[reuse];
      B.tzy[r] = B.tzy[reuse];
      continue;
    }
    CellDesc<T> D;
    std::memset(&D, 0, sizeof(D));
    fill_desc<T>(B, r, D);
    for (int axis = 0; axis < 2; ++axis) {
      if (axis == 0 ? B.mx[r] : B.my[r]) continue;  // two-step pass: the tile follows from the length
      const int nl = axis == 0 ? c.n[0] : c.n[1];
      float best = -1.f;
      int best_tz = 1;
      for (int tz : {2, 4, 8, 16, 32}) {
        if (tz > 2 * c.g.nh3 && tz > 2) continue;
        if ((size_t)(nl + 2 * nl * tz) * eb > 64 * 1024) continue;
        if (axis == 0 && nl * tz > 8 * 256) continue;  // register budget of the fused x modes
        const float ms = tune_strided_ms<T>(D, axis, tz, B.st, 3);
        if (ms > 0.f && (best < 0.f || ms < best)) {
          best = ms;
          best_tz = tz;
        }
      }
      (axis == 0 ? B.tzx : B.tzy)[r] = best_tz;
    }
  }
  HIPCK(hipGetLastError());
  for (int r = 0; r < n; ++r) {
    Ctx& c = *B.cells[r];
    const long long nlines = (long long)c.n[0] * c.n[1];
    if (B.mx[r]) {
      const int tz = B.tzx[r];
      bx[r + 1] = bx[r] + (int)(((long long)c.n[1] * c.g.nh3 + tz - 1) / tz);
      lx = std::max(lx, (size_t)(c.n[0] + (size_t)c.n[0] * (tz + 1)) * eb);
    } else {
      const int ntx = (c.g.nh3 + B.tzx[r] - 1) / B.tzx[r];
      bx[r + 1] = bx[r] + ntx * c.n[1];
      lx = std::max(lx, (size_t)(c.n[0] + 2 * c.n[0] * B.tzx[r]) * eb);
    }
    if (B.my[r]) {
      const int tz = B.tzy[r];
      by[r + 1] = by[r] + c.ncomp * (int)(((long long)c.n[0] * c.g.nh3 + tz - 1) / tz);
      ly = std::max(ly, (size_t)(c.n[1] + (size_t)c.n[1] * (tz + 1)) * eb);
    } else {
      const int nty = (c.g.nh3 + B.tzy[r] - 1) / B.tzy[r];
      by[r + 1] = by[r] + nty * c.n[0] * c.ncomp;
      ly = std::max(ly, (size_t)(c.n[1] + 2 * c.n[1] * B.tzy[r]) * eb);
    }
    const size_t M = c.g.n3 / 2;
    if (B.mz[r]) {
      const int tl = two_step_threads((int)M), lb = 64 / tl;
      // anisotropic or finite-strain tangents (FP32): one line group per
      // block, its components staged in LDS (mixed_line_staged)
      const bool staged = B.mz[r] == 2;
      const long long per_block = staged ? lb : (long long)(kLineThreads / 64) * lb;
      bz[r + 1] = bz[r] + (int)((nlines + per_block - 1) / per_block);
      if ((size_t)(bz[r + 1] - bz[r]) > c.npart) DB_THROW(DBFFT_EUNSUPPORTED, "z pass partials exceed the cell's buffer");
      lz = std::max(lz, (size_t)(2 * M + 1 + (size_t)(kLineThreads / 64) * lb * (M + tl + 1) +
                                 (staged ? (size_t)c.ncomp * lb * M : 0)) * eb);
    } else {
      bz[r + 1] = bz[r] + (int)((nlines + B.L[r] - 1) / B.L[r]);
      lz = std::max(lz, line_smem_bytes(c.g, B.L[r], c.ncomp, (int)eb));
    }
    bv[r + 1] = bv[r] + pcg_block_count(c.g);
  }
  std::vector<int> boff;
  boff.insert(boff.end(), bx.begin(), bx.end());
  boff.insert(boff.end(), by.begin(), by.end());
  boff.insert(boff.end(), bz.begin(), bz.end());
  boff.insert(boff.end(), bv.begin(), bv.end());
  B.boff_dev = static_cast<int*>(dalloc(boff.size() * sizeof(int)));
  HIPCK(hipMemcpy(B.boff_dev, boff.data(), boff.size() * sizeof(int), hipMemcpyHostToDevice));
  B.bl.ncell = n;
  B.bl.kin = B.kin;
  B.bl.law = (B.cells[0]->mat == DBFFT_MAT_SVK) ? 2 : 0;
  B.bl.ncomp = B.ncomp;
  B.bl.nbx_f = bx[n];
  B.bl.nby = by[n];
  B.bl.nbz = bz[n];
  B.bl.nbv = bv[n];
  B.bl.boff_xf = B.boff_dev;
  B.bl.boff_y = B.boff_dev + (n + 1);
  B.bl.boff_z = B.boff_dev + 2 * (n + 1);
  B.bl.boff_v = B.boff_dev + 3 * (n + 1);
  B.bl.lds_x = lx;
  B.bl.lds_y = ly;
  B.bl.lds_z = lz;
  B.bl.gen_x = B.bl.gen_y = B.bl.gen_z = 0;
  for (int r = 0; r < n; ++r) {
    if (!B.mx[r]) B.bl.gen_x = 1;
    if (!B.my[r]) B.bl.gen_y = 1;
    if (!B.mz[r]) B.bl.gen_z = 1;
  }
  B.desc_dev = dalloc(B.desc_host.size());
  B.flags_dev = static_cast<int*>(dalloc(n * sizeof(int)));
  HIPCK(hipHostMalloc((void**)&B.flags_host, n * sizeof(int), hipHostMallocDefault));
}

// descriptors with the current tangents and the per-cell preconditioners
template <typename T>
static void batch_upload(Batch& B, const std::vector<PrecondArgs>& pa, const std::vector<PcgConst>& pc) {
  const int n = (int)B.cells.size();
  for (int r = 0; r < n; ++r) {
    CellDesc<T>* D = reinterpret_cast<CellDesc<T>*>(B.desc_host.data() + r * B.desc_size);
    fill_desc<T>(B, r, *D);
    D->pa = pa[r];
    D->pc = pc[r];
  }
  HIPCK(hipMemcpyAsync(B.desc_dev, B.desc_host.data(), B.desc_host.size(), hipMemcpyHostToDevice, B.st));
  HIPCK(hipStreamSynchronize(B.st));
}

// batched PCG: cells with active[r] != 0 solve K x = b (b in their r);
// the others are marked converged and skipped by every kernel
// rho_prev (may be null): per cell, > 0 to go on with the direction in p
// after a residual replacement (pcg_resume) instead of starting from p = M r.
template <typename T>
static std::vector<PcgOut> batch_pcg(Batch& B, const std::vector<int>& active, const std::vector<PrecondArgs>& pa,
                                     const std::vector<PcgConst>& pc, const std::vector<std::array<double, 9>>& sig0,
                                     const std::vector<std::array<double, kMaxMacro>>& re0,
                                     const std::vector<double>* rho_prev = nullptr) {
  const int n = (int)B.cells.size();
  batch_upload<T>(B, pa, pc);
  for (int r = 0; r < n; ++r) {
    Ctx& c = *B.cells[r];
    if (active[r]) {
      const double rho = rho_prev ? (*rho_prev)[r] : 0.0;
      if (rho > 0.0) pcg_resume<T>(c, pa[r], pc[r], c.x, c.r, c.p, sig0[r].data(), re0[r].data(), rho);
      else pcg_begin<T>(c, pa[r], pc[r], c.x, c.r, c.p, sig0[r].data(), re0[r].data());
    } else {
      std::memset(c.sc_host, 0, sizeof(PcgScalars));
      c.sc_host->converged = 1;
      HIPCK(hipMemcpyAsync(c.sc_dev, c.sc_host, sizeof(PcgScalars), hipMemcpyHostToDevice, c.st));
      HIPCK(hipStreamSynchronize(c.st));
    }
  }
  auto all_done = [&]() {
    launch_batch_flags<T>(B.desc_dev, n, B.flags_dev, B.st);
    HIPCK(hipMemcpyAsync(B.flags_host, B.flags_dev, n * sizeof(int), hipMemcpyDeviceToHost, B.st));
    HIPCK(hipStreamSynchronize(B.st));
    for (int r = 0; r < n; ++r)
      if (!B.flags_host[r]) return false;
    return true;
  };
  if (B.use_graph && B.exec != nullptr && B.graph_chunk != B.chunk) {
    HIPCK(hipGraphExecDestroy(B.exec));
    HIPCK(hipGraphDestroy(B.graph));
    B.exec = nullptr;
    B.graph = nullptr;
  }
  if (B.use_graph && B.exec == nullptr) {
    B.graph_chunk = B.chunk;
    HIPCK(hipStreamBeginCapture(B.st, hipStreamCaptureModeThreadLocal));
    for (int k = 0; k < B.chunk; ++k) launch_batch_iteration<T>(B.bl, B.desc_dev, B.st);
    HIPCK(hipStreamEndCapture(B.st, &B.graph));
    HIPCK(hipGraphInstantiate(&B.exec, B.graph, nullptr, nullptr, 0));
  }
  while (!all_done()) {
    if (B.use_graph) {
      HIPCK(hipGraphLaunch(B.exec, B.st));
    } else {
      for (int k = 0; k < B.chunk; ++k) launch_batch_iteration<T>(B.bl, B.desc_dev, B.st);
    }
    HIPCK(hipGetLastError());
  }
  std::vector<PcgOut> out(n);
  for (int r = 0; r < n; ++r) {
    Ctx& c = *B.cells[r];
    HIPCK(hipMemcpyAsync(c.sc_host, c.sc_dev, sizeof(PcgScalars), hipMemcpyDeviceToHost, c.st));
    HIPCK(hipStreamSynchronize(c.st));
    out[r] = pcg_result(c);
  }
  return out;
}

template <typename T>
static std::vector<int> batch_solve_t(Batch& B, const double* loads, const uint8_t* masks, int ninc, double dt,
                                      const dbfft_opts& o, dbfft_info* infos) {
  const int n = (int)B.cells.size();
  std::vector<int> status(n, DBFFT_OK);
  std::vector<PrecondArgs> pa(n);
  std::vector<PcgConst> pc(n);
  std::vector<std::array<double, 9>> sig0(n);
  std::vector<std::array<double, kMaxMacro>> re0(n);
  std::vector<int> active(n, 0);
  B.chunk = std::max(1, o.check_every);
  const bool linear = B.cells[0]->linear_material();
  if (linear) {
    // single batched PCG per refinement step (one step in FP64)
    std::vector<MacroSet> ms(n);
    std::vector<std::array<double, kMaxMacro>> sbar(n), e(n), re_b(n);
    std::vector<std::array<double, 9>> dc0(n);
    std::vector<double> eqv(n, INFINITY), ldv(n, INFINITY);
    std::vector<double> rho_prev(n, 0.0), rec_eq(n, 0.0), rec_ld(n, 0.0);  // FP32_MIXED residual replacement
    std::vector<int> iters(n, 0), refine(n, 0), done(n, 0);
    for (int r = 0; r < n; ++r) {
      Ctx& c = *B.cells[r];
      int mask[9];
      for (int i = 0; i < 9; ++i) mask[i] = masks[9 * r + i] ? 1 : 0;
      for (int i = 0; i < 9; ++i) c.last_mask[i] = mask[i];
      ms[r] = macro_set(c, mask);
      double U_rm[9], lst[9];
      for (int i = 0; i < 9; ++i) U_rm[i] = mask[i] ? 0.0 : loads[9 * r + i];
      rm_to_stored(c.kin, U_rm, c.EU_st);
      rm_to_stored(c.kin, loads + 9 * r, lst);
      sbar[r].fill(0.0);
      e[r].fill(0.0);
      for (int a = 0; a < ms[r].nS; ++a) sbar[r][a] = bdot(c.kin, ms[r].bst[a], lst);
      double C4[81];
      mean_tangent(c, C4);
      std::memset(&pc[r], 0, sizeof(PcgConst));
      build_precond(c, C4, ms[r], pa[r], pc[r]);
      pc[r].tol = o.tol;
      pc[r].tol_load = o.tol_load;
      pc[r].max_iter = o.max_iter;
      TangentArgs<double> tan64 = elastic_tangent<double>(c);
      set_macro(c, c.EU_st);
      apply_const<double>(c, c.b, c.mac_dev, tan64, c.dc_dev);
      launch_axpby<double>(c.b, c.b, 0.0, -1.0, 6 * c.g.nh, c.st);
      double d0[9];
      read_dc(c, d0);
      for (int i = 0; i < 9; ++i) dc0[r][i] = d0[i];
      re_b[r].fill(0.0);
      for (int a = 0; a < ms[r].nS; ++a) re_b[r][a] = sbar[r][a] - bdot(c.kin, ms[r].bst[a], d0);
      HIPCK(hipMemsetAsync(c.sol, 0, 3 * (size_t)c.g.nh * 2 * sizeof(double), c.st));
      HIPCK(hipMemcpyAsync(c.t64, c.b, 3 * (size_t)c.g.nh * 2 * sizeof(double), hipMemcpyDeviceToDevice, c.st));
    }
    for (int step = 0;; ++step) {
      // residual of every unfinished cell (FP64), then one batched inner solve
      bool any = false;
      for (int r = 0; r < n; ++r) {
        active[r] = 0;
        if (done[r]) continue;
        Ctx& c = *B.cells[r];
        double sig[9];
        std::array<double, kMaxMacro> re = re_b[r];
        if (step == 0) {
          for (int i = 0; i < 9; ++i) sig[i] = dc0[r][i];
        } else {
          double mt[9] = {0};
          for (int a = 0; a < ms[r].nS; ++a)
            for (int k = 0; k < 9; ++k) mt[k] += e[r][a] * ms[r].bst[a][k];
          set_macro(c, mt);
          TangentArgs<double> tan64 = elastic_tangent<double>(c);
          apply_K<double>(c, c.sol, c.t64, c.mac_dev, nullptr, tan64, c.partA, c.dc_dev, nullptr);
          launch_axpby<double>(c.t64, c.b, 1.0, -1.0, 6 * c.g.nh, c.st);
          double dcx[9];
          read_dc(c, dcx);
          for (int i = 0; i < 9; ++i) sig[i] = dc0[r][i] + dcx[i];
          for (int a = 0; a < ms[r].nS; ++a) re[a] = re_b[r][a] - bdot(c.kin, ms[r].bst[a], dcx);
        }
        const double nrm = frob_stored(c.kin, sig);
        const double ra = std::sqrt(std::max(dot64(c, c.t64, c.t64), 0.0));
        double rl = 0.0;
        for (int a = 0; a < ms[r].nS; ++a) rl += re[a] * re[a];
        rl = std::sqrt(rl);
        eqv[r] = nrm > 0 ? ra / nrm : (ra == 0 ? 0.0 : INFINITY);
        ldv[r] = nrm > 0 ? rl / nrm : (rl == 0 ? 0.0 : INFINITY);
        // as in the single-cell solve: keep the direction only while the
        // FP32 recursion tracked the true residual within a factor of 10
        if (rho_prev[r] > 0.0 &&
            (eqv[r] > 10.0 * rec_eq[r] || ldv[r] > 10.0 * std::max(rec_ld[r], 0.1 * o.tol_load)))
          rho_prev[r] = 0.0;
        if (eqv[r] < o.tol && ldv[r] < o.tol_load) {
          done[r] = 1;
          status[r] = DBFFT_OK;
          continue;
        }
        if (refine[r] >= o.max_refine || iters[r] >= o.max_iter) {
          done[r] = 1;
          status[r] = DBFFT_ENOTCONV;
          continue;
        }
        PcgConst pci = pc[r];
        if (B.prec != DBFFT_FP64) {
          pci.tol = std::max(eqv[r] * o.inner_tol, 0.5 * o.tol);
          pci.tol_load = std::max(ldv[r] * o.inner_tol, 0.5 * o.tol_load);
        }
        pci.max_iter = std::max(1, o.max_iter - iters[r]);
        pc[r] = pci;
        for (int i = 0; i < 9; ++i) sig0[r][i] = sig[i];
        re0[r] = re;
        if (B.prec == DBFFT_FP64)
          HIPCK(hipMemcpyAsync(c.r, c.t64, 3 * (size_t)c.g.nh * 2 * sizeof(double), hipMemcpyDeviceToDevice, c.st));
        else
          launch_convert<double, float>(c.r, c.t64, 6 * c.g.nh, c.st);
        active[r] = 1;
        any = true;
      }
      if (!any) break;
      std::vector<PcgOut> po = batch_pcg<T>(B, active, pa, pc, sig0, re0, &rho_prev);
      for (int r = 0; r < n; ++r) {
        if (!active[r]) continue;
        Ctx& c = *B.cells[r];
        iters[r] += po[r].iters;
        refine[r] += (B.prec == DBFFT_FP64) ? 0 : 1;
        if (po[r].status == 2) {
          status[r] = DBFFT_EBREAKDOWN;
          done[r] = 1;
          continue;
        }
        if (B.prec != DBFFT_FP64) {
          const PcgScalars& hs = *c.sc_host;
          rho_prev[r] = (po[r].status == 1 && hs.beta > 0.0 && hs.rz > 0.0) ? hs.rz / hs.beta : 0.0;
          rec_eq[r] = po[r].eq;
          rec_ld[r] = po[r].ld;
        }
        if (B.prec == DBFFT_FP64) {
          // FP64: one PCG solves the system; its recurrence decides the status
          HIPCK(hipMemcpyAsync(c.sol, c.x, 3 * (size_t)c.g.nh * 2 * sizeof(double), hipMemcpyDeviceToDevice, c.st));
          for (int a = 0; a < ms[r].nS; ++a) e[r][a] += po[r].xe[a];
          status[r] = pcg_status(po[r].status);
          done[r] = 1;
          continue;
        } else {
          launch_convert<float, double>(c.q, c.x, 6 * c.g.nh, c.st);
          launch_axpby<double>(c.sol, c.q, 1.0, 1.0, 6 * c.g.nh, c.st);
        }
        for (int a = 0; a < ms[r].nS; ++a) e[r][a] += po[r].xe[a];
      }
    }
    for (int r = 0; r < n; ++r) {
      Ctx& c = *B.cells[r];
      for (int i = 0; i < 9; ++i) c.e_st[i] = 0.0;
      for (int a = 0; a < ms[r].nS; ++a)
        for (int i = 0; i < 9; ++i) c.e_st[i] += e[r][a] * ms[r].bst[a][i];
      double mt[9], sig_st[9], eq, ld;
      for (int i = 0; i < 9; ++i) mt[i] = c.EU_st[i] + c.e_st[i];
      evaluate_linear(c, c.sol, mt, ms[r], sbar[r].data(), sig_st, eq, ld);
      stored_to_rm(c.kin, sig_st, c.sig_rm);
      stored_to_rm(c.kin, mt, c.eps_rm);
      c.solved = true;
      c.ck_n = 0;
      dbfft_info& inf = infos[r];
      std::memset(&inf, 0, sizeof(inf));
      inf.pcg_iters = iters[r];
      inf.refine_steps = refine[r];
      inf.increments = 1;
      inf.eq_res = eq;
      inf.load_res = ld;
      inf.status = status[r];
      for (int i = 0; i < 9; ++i) {
        inf.sigma_bar[i] = c.sig_rm[i];
        inf.eps_bar[i] = c.eps_rm[i];
      }
    }
    return status;
  }

  // Newton in lockstep: every unfinished cell evaluates its residual, then
  // one batched PCG solves all linear corrections
  std::vector<NewtonState> S(n);
  for (int r = 0; r < n; ++r) {
    Ctx& c = *B.cells[r];
    int mask[9];
    for (int i = 0; i < 9; ++i) mask[i] = masks[9 * r + i] ? 1 : 0;
    for (int i = 0; i < 9; ++i) c.last_mask[i] = mask[i];
    newton_init(c, S[r], loads + 9 * r, mask, ninc, dt, o);
  }
  for (int k = 1; k <= ninc; ++k) {
    std::vector<int> inc_done(n, 0);
    for (int r = 0; r < n; ++r) {
      if (S[r].status != DBFFT_OK) {
        inc_done[r] = 1;
        continue;
      }
      newton_begin_increment(*B.cells[r], S[r], k);
    }
    for (;;) {
      bool any = false;
      for (int r = 0; r < n; ++r) {
        active[r] = 0;
        if (inc_done[r]) continue;
        const int ev = newton_evaluate(*B.cells[r], S[r]);
        if (ev == 1) {
          inc_done[r] = 1;
          newton_end_increment(*B.cells[r], S[r]);
          continue;
        }
        if (ev < 0) {
          S[r].status = DBFFT_ENOTCONV;
          inc_done[r] = 1;
          continue;
        }
        pa[r] = S[r].pa;
        pc[r] = S[r].pc;
        for (int i = 0; i < 9; ++i) sig0[r][i] = S[r].sig_st[i];
        for (int a = 0; a < kMaxMacro; ++a) re0[r][a] = S[r].re[a];
        active[r] = 1;
        any = true;
      }
      if (!any) break;
      std::vector<PcgOut> po = batch_pcg<T>(B, active, pa, pc, sig0, re0);
      for (int r = 0; r < n; ++r) {
        if (!active[r]) continue;
        newton_apply_correction(*B.cells[r], S[r], po[r]);
        if (S[r].status != DBFFT_OK) inc_done[r] = 1;
      }
    }
  }
  for (int r = 0; r < n; ++r) {
    Ctx& c = *B.cells[r];
    newton_finish(c, S[r]);
    c.solved = true;
    infos[r] = S[r].info;
    status[r] = S[r].status;
  }
  return status;
}

static void batch_release(Batch* B) {
  if (B->st) (void)hipStreamSynchronize(B->st);
  if (B->exec) (void)hipGraphExecDestroy(B->exec);
  if (B->graph) (void)hipGraphDestroy(B->graph);
  if (B->desc_dev) (void)hipFree(B->desc_dev);
  if (B->boff_dev) (void)hipFree(B->boff_dev);
  if (B->flags_dev) (void)hipFree(B->flags_dev);
  if (B->flags_host) (void)hipHostFree(B->flags_host);
  if (B->st) (void)hipStreamDestroy(B->st);
  for (hipStream_t s : B->lane_st) (void)hipStreamDestroy(s);
}

// ------------------------------------------------------------------ allocation-free apply
// dbfft_apply_noalloc keeps everything beyond the caller's inputs and
// outputs in this array: twiddle tables, the spectral workspace (6 + 3 + 3
// half-spectrum components), partial sums, the macro block, a status word
// and a checked copy of the phase map.  Every GPU the library runs on holds
// its own copy until the process ends; host code reaches it only through
// the address hipGetSymbolAddress gives on that device (the array's name
// is a host-side stand-in there, not a device address).
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxScratchDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxScratchDevices] = {nullptr};

// device address of `scratch` on the current device, looked up once per device
static unsigned char* scratch_on_current_device() {
  int dev = 0;
  HIPCK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxScratchDevices) DB_THROW(DBFFT_EUNSUPPORTED, "device index above 63");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[dev] == nullptr) {
    void* ptr = nullptr;
    HIPCK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (ptr == nullptr) DB_THROW(DBFFT_EHIP, "hipGetSymbolAddress returned a null scratch address");
    g_scratch_ptr[dev] = ptr;
  }
  return static_cast<unsigned char*>(g_scratch_ptr[dev]);
}

// Twiddle tables w(k) = exp(-2 pi i k / denom), k < count, of the four
// transform axes (the values the context tables hold, computed on the
// device), and zeros over the macro block, the DC output and the status word.
struct TwiddleSegs {
  double* p[4];
  int denom[4];
  int count[4];
};

__global__ void k_noalloc_init(TwiddleSegs ts, double* zero, int nzero) {
  const int gid = blockIdx.x * blockDim.x + threadIdx.x, gs = gridDim.x * blockDim.x;
  for (int a = 0; a < 4; ++a)
    for (int k = gid; k < ts.count[a]; k += gs) {
      double sn, cs;
      sincospi(2.0 * (double)k / (double)ts.denom[a], &sn, &cs);
      ts.p[a][2 * k] = cs;
      ts.p[a][2 * k + 1] = -sn;
    }
  for (int i = gid; i < nzero; i += gs) zero[i] = 0.0;
}

// copy of the phase map with out-of-range ids replaced by 0 and flagged
__global__ void k_noalloc_phase(const uint8_t* __restrict__ in, uint8_t* __restrict__ out, long long n, int nphase,
                                int* __restrict__ bad) {
  int seen = 0;
  for (long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (long long)gridDim.x * blockDim.x) {
    uint8_t ph = in[v];
    if (ph >= nphase) {
      ph = 0;
      seen = 1;
    }
    out[v] = ph;
  }
  if (seen) *bad = 1;
}

// NaN over the output when the phase check flagged an id
__global__ void k_noalloc_poison(double* __restrict__ f, long long n, const int* __restrict__ bad) {
  if (*bad == 0) return;
  const double nan = __builtin_nan("");
  for (long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (long long)gridDim.x * blockDim.x)
    f[v] = nan;
}

// Carves the scratch array for one grid: returns the bytes needed and, when
// `base` is not null, sets the context's tables and workspaces to point into it.
struct NoallocLayout {
  double* zero;      // macro block (16), DC output (16), status word (as int)
  int nzero;
  uint8_t* phase;
  size_t bytes;
};

static NoallocLayout noalloc_layout(Ctx& c, unsigned char* base, bool phase_copy) {
  size_t off = 0;
  auto take = [&](size_t nbytes) -> unsigned char* {
    unsigned char* p = base ? base + off : nullptr;
    off += (nbytes + 255) / 256 * 256;
    return p;
  };
  const Geom& g = c.g;
  const int Z = z_length(g.n3), M = g.n3 / 2;
  c.td.tw1 = take((size_t)g.n1 * 16);
  c.td.tw2 = take((size_t)g.n2 * 16);
  c.td.tw3 = take((size_t)std::max(Z, 1) * 16);
  c.td.rtw = take((size_t)(M + 1) * 16);
  NoallocLayout L;
  L.nzero = 40;
  L.zero = reinterpret_cast<double*>(take((size_t)L.nzero * sizeof(double)));
  c.mac_dev = L.zero;
  c.dc_dev = L.zero ? L.zero + 16 : nullptr;
  c.npart = (size_t)partial_count(g);
  c.partA = reinterpret_cast<double*>(take(c.npart * sizeof(double)));
  L.phase = phase_copy ? take((size_t)g.nvox) : nullptr;
  const size_t vb = 3 * (size_t)g.nh * 2 * sizeof(double);
  c.W = take(2 * vb);
  c.p = take(vb);
  c.q = take(vb);
  L.bytes = off;
  return L;
}

}  // namespace dbfft

using namespace dbfft;

struct dbfft_ctx {
  Ctx impl;
};

static Ctx* C(dbfft_ctx* c) { return &c->impl; }

#define API_BEGIN try {
#define API_END                                       \
  }                                                   \
  catch (const Err& e) {                              \
    return (dbfft_status)e.code;                      \
  }                                                   \
  catch (...) {                                       \
    g_err = "unexpected C++ exception";               \
    return DBFFT_EHIP;                                \
  }

extern "C" {

void dbfft_default_opts(dbfft_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->tol = 1e-8;
  o->tol_load = 1e-10;
  o->max_iter = 10000;
  o->newton_tol = 1e-6;
  o->max_newton = 25;
  o->refresh = 0;
  o->inner_tol = 1e-2;
  o->max_refine = 30;
  o->check_every = 8;
  o->fused_cg = 1;
  o->graph = 1;
}

const char* dbfft_last_error(void) { return g_err.c_str(); }

dbfft_status dbfft_kernel_timing(dbfft_ctx* ctx, int32_t enable, double ms_total[16], int64_t launches[16]) {
  g_err.clear();
  API_BEGIN
  if (!ctx) DB_THROW(DBFFT_EINVAL, "null context");
  Ctx& c = *C(ctx);
  if (ms_total)
    for (int k = 0; k < 16; ++k) ms_total[k] = c.prof_ms[k];
  if (launches)
    for (int k = 0; k < 16; ++k) launches[k] = c.prof_n[k];
  if (enable && !c.prof_on) {
    for (int k = 0; k < 16; ++k) {
      c.prof_ms[k] = 0.0;
      c.prof_n[k] = 0;
    }
  }
  c.prof_on = enable ? 1 : 0;
  return DBFFT_OK;
  API_END
}

dbfft_status dbfft_setup(dbfft_ctx** out, const int64_t n[3], int32_t kinematics, int32_t precision, int32_t material,
                         const void* field_dev, const double* params, int32_t nparams, void* hip_stream) {
  g_err.clear();
  API_BEGIN
  if (!out) DB_THROW(DBFFT_EINVAL, "null output pointer");
  *out = nullptr;
  dbfft_ctx* h = new dbfft_ctx();
  try {
    setup(&h->impl, n, kinematics, precision, material, field_dev, params, nparams, hip_stream);
  } catch (...) {
    release(&h->impl);
    delete h;
    throw;
  }
  *out = h;
  return DBFFT_OK;
  API_END
}

void dbfft_destroy(dbfft_ctx* ctx) {
  if (!ctx) return;
  release(&ctx->impl);
  delete ctx;
}

dbfft_status dbfft_apply(dbfft_ctx* ctx, const double* u_dev, double* f_dev) {
  g_err.clear();
  API_BEGIN
  if (!ctx || !u_dev || !f_dev) DB_THROW(DBFFT_EINVAL, "null argument");
  Ctx& c = *C(ctx);
  const StridedGeom sx = xgeom(c), sy = ygeom(c);
  const long long N = c.g.nvox;
  double zero[9] = {0};
  set_macro(c, zero);
  if (c.prec == DBFFT_FP64) {
    Tables<double>& tb = c.td;
    TangentArgs<double> tan = elastic_tangent<double>(c);
    launch_line<double>(LP_R2C, c.kin, u_dev, c.W, c.g, c.p3, tb.tw3, tb.rtw, tan, nullptr, nullptr, nullptr, 3,
                        c.st, nullptr, nullptr);
    launch_strided<double>(SP_PLAIN, c.W, c.W, 3, sy, c.g, c.p2, tb.tw2, -1, nullptr, c.st, nullptr);
    launch_strided<double>(SP_PLAIN, c.W, c.p, 3, sx, c.g, c.p1, tb.tw1, -1, nullptr, c.st, nullptr);
    apply_K<double>(c, c.p, c.q, c.mac_dev, nullptr, tan, c.partA, c.dc_dev, nullptr);
    launch_strided<double>(SP_PLAIN, c.q, c.W, 3, sx, c.g, c.p1, tb.tw1, +1, nullptr, c.st, nullptr);
    launch_strided<double>(SP_PLAIN, c.W, c.W, 3, sy, c.g, c.p2, tb.tw2, +1, nullptr, c.st, nullptr);
    launch_line<double>(LP_C2R, c.kin, c.W, f_dev, c.g, c.p3, tb.tw3, tb.rtw, tan, nullptr, nullptr, nullptr, 3,
                        c.st, nullptr, nullptr);
  } else {
    Tables<float>& tb = c.tf;
    TangentArgs<float> tan = elastic_tangent<float>(c);
    float* u32 = reinterpret_cast<float*>(c.fa);
    launch_convert<double, float>(u32, u_dev, 3 * N, c.st);
    launch_line<float>(LP_R2C, c.kin, u32, c.W, c.g, c.p3, tb.tw3, tb.rtw, tan, nullptr, nullptr, nullptr, 3, c.st,
                       nullptr, nullptr);
    launch_strided<float>(SP_PLAIN, c.W, c.W, 3, sy, c.g, c.p2, tb.tw2, -1, nullptr, c.st, nullptr);
    launch_strided<float>(SP_PLAIN, c.W, c.p, 3, sx, c.g, c.p1, tb.tw1, -1, nullptr, c.st, nullptr);
    apply_K<float>(c, c.p, c.q, c.mac_dev, nullptr, tan, c.partA, c.dc_dev, nullptr);
    launch_strided<float>(SP_PLAIN, c.q, c.W, 3, sx, c.g, c.p1, tb.tw1, +1, nullptr, c.st, nullptr);
    launch_strided<float>(SP_PLAIN, c.W, c.W, 3, sy, c.g, c.p2, tb.tw2, +1, nullptr, c.st, nullptr);
    launch_line<float>(LP_C2R, c.kin, c.W, u32, c.g, c.p3, tb.tw3, tb.rtw, tan, nullptr, nullptr, nullptr, 3, c.st,
                       nullptr, nullptr);
    launch_convert<float, double>(f_dev, u32, 3 * N, c.st);
  }
  HIPCK(hipGetLastError());
  HIPCK(hipStreamSynchronize(c.st));
  return DBFFT_OK;
  API_END
}

dbfft_status dbfft_apply_noalloc(const int64_t n[3], int32_t material, const void* field_dev, const double* params,
                                 int32_t nparams, const double* u_dev, double* f_dev, void* hip_stream) {
  g_err.clear();
  API_BEGIN
  if (!n || !field_dev || !params || !u_dev || !f_dev) DB_THROW(DBFFT_EINVAL, "null argument");
  check_grid(n, DBFFT_SMALL);
  if (material != DBFFT_MAT_ISO_PHASE && material != DBFFT_MAT_ISO_FIELD)
    DB_THROW(DBFFT_EUNSUPPORTED, "dbfft_apply_noalloc takes ISO_PHASE or ISO_FIELD materials");
  if (nparams < 1) DB_THROW(DBFFT_EINVAL, "null material parameters");
  Ctx c;
  init_grid(&c, n, DBFFT_SMALL, DBFFT_FP64, material, hip_stream);
  TangentArgs<double> tan;
  std::memset(&tan, 0, sizeof(tan));
  if (material == DBFFT_MAT_ISO_PHASE) {
    tan.kind = TAN_ISO_PHASE;
    iso_phase_table(params, nparams, tan.nphase, tan.lam, tan.mu);
  } else {
    tan.kind = TAN_ISO_FIELD;
    const double nu = params[0];
    tan.lam1 = nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
    tan.mu1 = 1.0 / (2.0 * (1.0 + nu));
    tan.field = static_cast<const double*>(field_dev);
  }
  const bool by_phase = material == DBFFT_MAT_ISO_PHASE;
  const size_t need = noalloc_layout(c, nullptr, by_phase).bytes;
  if (need > kScratchBytes)
    DB_THROW(DBFFT_EUNSUPPORTED, "grid needs " + std::to_string(need) + " bytes of device scratch, above the " +
                                     std::to_string(kScratchBytes) +
                                     " bytes dbfft_apply_noalloc holds; use dbfft_setup and dbfft_apply");
  unsigned char* base = scratch_on_current_device();
  const NoallocLayout L = noalloc_layout(c, base, by_phase);
  const Geom& g = c.g;
  const long long N = g.nvox;
  int* bad = reinterpret_cast<int*>(L.zero + 32);
  TwiddleSegs ts;
  const int Z = z_length(g.n3), M = g.n3 / 2;
  const void* tabs[4] = {c.td.tw1, c.td.tw2, c.td.tw3, c.td.rtw};
  const int denom[4] = {g.n1, g.n2, std::max(Z, 1), g.n3}, count[4] = {g.n1, g.n2, std::max(Z, 1), M + 1};
  for (int a = 0; a < 4; ++a) {
    ts.p[a] = static_cast<double*>(const_cast<void*>(tabs[a]));
    ts.denom[a] = denom[a];
    ts.count[a] = count[a];
  }
  hipLaunchKernelGGL(k_noalloc_init, dim3(16), dim3(256), 0, c.st, ts, L.zero, L.nzero);
  const int vb = (int)std::min<long long>((N + 255) / 256, 2048);
  if (by_phase) {
    hipLaunchKernelGGL(k_noalloc_phase, dim3(vb), dim3(256), 0, c.st, static_cast<const uint8_t*>(field_dev),
                       L.phase, N, tan.nphase, bad);
    tan.phase = L.phase;
  }
  const StridedGeom sx = xgeom(c), sy = ygeom(c);
  Tables<double>& tb = c.td;
  launch_line<double>(LP_R2C, c.kin, u_dev, c.W, g, c.p3, tb.tw3, tb.rtw, tan, nullptr, nullptr, nullptr, 3, c.st,
                      nullptr, nullptr);
  launch_strided<double>(SP_PLAIN, c.W, c.W, 3, sy, g, c.p2, tb.tw2, -1, nullptr, c.st, nullptr);
  launch_strided<double>(SP_PLAIN, c.W, c.p, 3, sx, g, c.p1, tb.tw1, -1, nullptr, c.st, nullptr);
  apply_K<double>(c, c.p, c.q, c.mac_dev, nullptr, tan, c.partA, c.dc_dev, nullptr);
  launch_strided<double>(SP_PLAIN, c.q, c.W, 3, sx, g, c.p1, tb.tw1, +1, nullptr, c.st, nullptr);
  launch_strided<double>(SP_PLAIN, c.W, c.W, 3, sy, g, c.p2, tb.tw2, +1, nullptr, c.st, nullptr);
  launch_line<double>(LP_C2R, c.kin, c.W, f_dev, g, c.p3, tb.tw3, tb.rtw, tan, nullptr, nullptr, nullptr, 3, c.st,
                      nullptr, nullptr);
  if (by_phase) hipLaunchKernelGGL(k_noalloc_poison, dim3(vb), dim3(256), 0, c.st, f_dev, 3 * N, bad);
  HIPCK(hipGetLastError());
  return DBFFT_OK;
  API_END
}

dbfft_status dbfft_apply_fourier(dbfft_ctx* ctx, const void* a_dev, const double* e_macro, void* f_dev,
                                 double* sigma_bar_out) {
  g_err.clear();
  API_BEGIN
  if (!ctx || !a_dev || !f_dev) DB_THROW(DBFFT_EINVAL, "null argument");
  Ctx& c = *C(ctx);
  double st[9] = {0};
  if (e_macro) rm_to_stored(c.kin, e_macro, st);
  set_macro(c, st);
  const long long n2 = 6 * c.g.nh;
  if (c.prec == DBFFT_FP64) {
    TangentArgs<double> tan = elastic_tangent<double>(c);
    apply_K<double>(c, a_dev, f_dev, c.mac_dev, nullptr, tan, c.partA, c.dc_dev, nullptr);
  } else {
    TangentArgs<float> tan = elastic_tangent<float>(c);
    launch_convert<double, float>(c.p, a_dev, n2, c.st);
    apply_K<float>(c, c.p, c.q, c.mac_dev, nullptr, tan, c.partA, c.dc_dev, nullptr);
    launch_convert<float, double>(f_dev, c.q, n2, c.st);
  }
  HIPCK(hipGetLastError());
  double dc[9];
  read_dc(c, dc);
  if (sigma_bar_out) stored_to_rm(c.kin, dc, sigma_bar_out);
  return DBFFT_OK;
  API_END
}

dbfft_status dbfft_solve(dbfft_ctx* ctx, const double load[9], const uint8_t stress_mask[9], int32_t n_increments,
                         double dt, const dbfft_opts* opts, dbfft_info* info) {
  g_err.clear();
  API_BEGIN
  if (!ctx || !load || !stress_mask) DB_THROW(DBFFT_EINVAL, "null argument");
  Ctx& c = *C(ctx);
  dbfft_opts o;
  if (opts) o = *opts;
  else dbfft_default_opts(&o);
  c.use_fused = o.fused_cg != 0;
  c.use_graph = o.graph != 0;
  if (o.coarse_kc != 0) DB_THROW(DBFFT_EUNSUPPORTED, "opts.coarse_kc applies to dbfft_solve_block");
  int mask[9];
  for (int i = 0; i < 9; ++i) mask[i] = stress_mask[i] ? 1 : 0;
  if (c.kin == KIN_SMALL) {
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        if (mask[i * 3 + j] != mask[j * 3 + i]) DB_THROW(DBFFT_EINVAL, "small strains need a symmetric stress mask");
        if (load[i * 3 + j] != load[j * 3 + i]) DB_THROW(DBFFT_EINVAL, "small strains need a symmetric load");
      }
  }
  dbfft_info inf;
  std::memset(&inf, 0, sizeof(inf));
  for (int i = 0; i < 9; ++i) c.last_mask[i] = mask[i];
  int status;
  if (c.linear_material()) {
    const MacroSet ms = macro_set(c, mask);
    double U_rm[9], lst[9];
    for (int i = 0; i < 9; ++i) U_rm[i] = mask[i] ? 0.0 : load[i];
    rm_to_stored(c.kin, U_rm, c.EU_st);
    rm_to_stored(c.kin, load, lst);
    double sbar[kMaxMacro] = {0};
    for (int a = 0; a < ms.nS; ++a) sbar[a] = bdot(c.kin, ms.bst[a], lst);
    LinOut lo = linear_solve(c, c.EU_st, ms, sbar, o, c.sol);
    status = lo.status;
    for (int i = 0; i < 9; ++i) c.e_st[i] = 0.0;
    for (int a = 0; a < ms.nS; ++a)
      for (int i = 0; i < 9; ++i) c.e_st[i] += lo.e_coef[a] * ms.bst[a][i];
    double mt[9], sig_st[9], eq, ld;
    for (int i = 0; i < 9; ++i) mt[i] = c.EU_st[i] + c.e_st[i];
    evaluate_linear(c, c.sol, mt, ms, sbar, sig_st, eq, ld);
    stored_to_rm(c.kin, sig_st, c.sig_rm);
    stored_to_rm(c.kin, mt, c.eps_rm);
    inf.pcg_iters = lo.iters;
    inf.refine_steps = lo.refine;
    inf.increments = 1;
    inf.eq_res = eq;
    inf.load_res = ld;
    for (int i = 0; i < 9; ++i) {
      inf.sigma_bar[i] = c.sig_rm[i];
      inf.eps_bar[i] = c.eps_rm[i];
    }
  } else {
    if (n_increments < 1) DB_THROW(DBFFT_EINVAL, "n_increments must be >= 1");
    if (c.mat == DBFFT_MAT_J2VP_CUBIC && !(dt > 0.0)) DB_THROW(DBFFT_EINVAL, "dt must be > 0 for J2VP_CUBIC");
    status = newton_solve(c, load, mask, n_increments, dt, o, inf);
  }
  inf.status = status;
  c.solved = true;
  if (info) *info = inf;
  if (status != DBFFT_OK && g_err.empty())
    g_err = status == DBFFT_ENOTCONV ? "iteration cap reached" : "breakdown: <p, K p> <= 0 or NaN";
  return (dbfft_status)status;
  API_END
}

dbfft_status dbfft_solve_block(dbfft_ctx* ctx, int32_t nrhs, const double* loads, const uint8_t stress_mask[9],
                               const dbfft_opts* opts, dbfft_info* infos, int32_t* applies) {
  g_err.clear();
  API_BEGIN
  if (!ctx || !loads || !stress_mask || !infos) DB_THROW(DBFFT_EINVAL, "null argument");
  Ctx& c = *C(ctx);
  if (nrhs < 1 || nrhs > kMaxBlock) DB_THROW(DBFFT_EINVAL, "nrhs must be 1 .. 6");
  if (!c.linear_material()) DB_THROW(DBFFT_EUNSUPPORTED, "block solves take linear materials");
  if (c.prec != DBFFT_FP64) DB_THROW(DBFFT_EUNSUPPORTED, "block solves run in FP64");
  dbfft_opts o;
  if (opts) o = *opts;
  else dbfft_default_opts(&o);
  int mask[9];
  for (int i = 0; i < 9; ++i) mask[i] = stress_mask[i] ? 1 : 0;
  if (c.kin == KIN_SMALL) {
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        if (mask[i * 3 + j] != mask[j * 3 + i]) DB_THROW(DBFFT_EINVAL, "small strains need a symmetric stress mask");
        for (int r = 0; r < nrhs; ++r)
          if (loads[9 * r + i * 3 + j] != loads[9 * r + j * 3 + i])
            DB_THROW(DBFFT_EINVAL, "small strains need symmetric loads");
      }
  }
  const BlockOut bo = block_solve(c, nrhs, loads, mask, o, infos);
  if (applies) *applies = bo.applies;
  if (bo.status != DBFFT_OK && g_err.empty())
    g_err = bo.status == DBFFT_ENOTCONV ? "iteration cap reached" : "breakdown: block <P, K P> not positive definite";
  return (dbfft_status)bo.status;
  API_END
}

dbfft_status dbfft_homogenize(dbfft_ctx* ctx, double sigma_bar[9], double eps_bar[9], double* strain_dev,
                              double* stress_dev, double* disp_dev) {
  g_err.clear();
  API_BEGIN
  if (!ctx) DB_THROW(DBFFT_EINVAL, "null context");
  Ctx& c = *C(ctx);
  if (!c.solved) DB_THROW(DBFFT_EINVAL, "no solution yet");
  if (sigma_bar)
    for (int i = 0; i < 9; ++i) sigma_bar[i] = c.sig_rm[i];
  if (eps_bar)
    for (int i = 0; i < 9; ++i) eps_bar[i] = c.eps_rm[i];
  double mt[9];
  for (int i = 0; i < 9; ++i) mt[i] = c.EU_st[i] + c.e_st[i];
  if (strain_dev) {
    set_macro(c, mt);
    strain_field(c, c.sol, c.mac_dev, strain_dev);
  }
  if (stress_dev) {
    if (c.linear_material()) {
      set_macro(c, mt);
      strain_field(c, c.sol, c.mac_dev, stress_dev, 1);
    } else {
      HIPCK(hipMemcpyAsync(stress_dev, c.fc, (size_t)c.ncomp * c.g.nvox * sizeof(double), hipMemcpyDeviceToDevice, c.st));
    }
  }
  if (disp_dev) {
    const StridedGeom sx = xgeom(c), sy = ygeom(c);
    Tables<double>& tb = c.td;
    TangentArgs<double> tan = elastic_tangent<double>(c);
    launch_strided<double>(SP_PLAIN, c.sol, c.W, 3, sx, c.g, c.p1, tb.tw1, +1, nullptr, c.st, nullptr);
    launch_strided<double>(SP_PLAIN, c.W, c.W, 3, sy, c.g, c.p2, tb.tw2, +1, nullptr, c.st, nullptr);
    launch_line<double>(LP_C2R, c.kin, c.W, disp_dev, c.g, c.p3, tb.tw3, tb.rtw, tan, nullptr, nullptr, nullptr, 3,
                        c.st, nullptr, nullptr);
  }
  HIPCK(hipGetLastError());
  HIPCK(hipStreamSynchronize(c.st));
  return DBFFT_OK;
  API_END
}

dbfft_status dbfft_solve_many(dbfft_ctx* ctx, int32_t nrhs, const double* loads, const uint8_t stress_mask[9],
                              const dbfft_opts* opts, dbfft_info* infos, int32_t nstreams) {
  g_err.clear();
  API_BEGIN
  if (!ctx || !loads || !stress_mask || !infos) DB_THROW(DBFFT_EINVAL, "null argument");
  if (nrhs < 1) DB_THROW(DBFFT_EINVAL, "nrhs must be at least 1");
  if (nstreams < 1 || nstreams > kMaxSolveStreams) DB_THROW(DBFFT_EINVAL, "nstreams must be 1 .. 8");
  Ctx& c = *C(ctx);
  if (!c.linear_material()) DB_THROW(DBFFT_EUNSUPPORTED, "dbfft_solve_many takes linear materials");
  if (opts && opts->coarse_kc != 0) DB_THROW(DBFFT_EUNSUPPORTED, "opts.coarse_kc applies to dbfft_solve_block");
  HIPCK(hipStreamSynchronize(c.st));
  const int ns = std::min<int>(nstreams, nrhs);
  // helper contexts: the same grid, precision and material (the field is
  // copied from this context's device copy), each on a stream of its own
  while ((int)c.helpers.size() < ns) {
    const void* field = (c.mat == DBFFT_MAT_ISO_PHASE) ? static_cast<const void*>(c.phase)
                        : (c.mat == DBFFT_MAT_ISO_FIELD) ? static_cast<const void*>(c.E64)
                                                         : static_cast<const void*>(c.grain);
    const int64_t n64[3] = {c.n[0], c.n[1], c.n[2]};
    hipStream_t s = nullptr;
    HIPCK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    dbfft_ctx* h = nullptr;
    const dbfft_status st = dbfft_setup(&h, n64, c.kin, c.prec, c.mat, field, c.setup_params.data(),
                                        (int32_t)c.setup_params.size(), s);
    if (st != DBFFT_OK) {
      const std::string m = dbfft_last_error();
      (void)hipStreamDestroy(s);
      DB_THROW(st, "helper context: " + m);
    }
    c.helpers.push_back(h);
    c.helper_streams.push_back(s);
  }
  const double len[3] = {1.0 / c.g.il1, 1.0 / c.g.il2, 1.0 / c.g.il3};
  for (int t = 0; t < ns; ++t) {
    const Geom& hg = C(c.helpers[t])->g;
    if (hg.il1 != c.g.il1 || hg.il2 != c.g.il2 || hg.il3 != c.g.il3) {
      const dbfft_status st = dbfft_set_lengths(c.helpers[t], len);
      if (st != DBFFT_OK) DB_THROW(st, std::string("helper context: ") + dbfft_last_error());
    }
  }
  // load j runs on helper j mod ns, each helper's loads in order on its own
  // host thread (contexts may be driven from different threads at once)
  std::vector<int> status(nrhs, DBFFT_OK);
  std::vector<std::string> msg(nrhs);
  std::vector<std::thread> th;
  th.reserve(ns);
  for (int t = 0; t < ns; ++t) {
    th.emplace_back([&, t]() {
      if (hipSetDevice(c.dev) != hipSuccess) {
        for (int j = t; j < nrhs; j += ns) {
          status[j] = DBFFT_EHIP;
          msg[j] = "hipSetDevice failed in a solve thread";
        }
        return;
      }
      for (int j = t; j < nrhs; j += ns) {
        status[j] = dbfft_solve(c.helpers[t], loads + 9 * (size_t)j, stress_mask, 1, 1.0, opts, &infos[j]);
        if (status[j] != DBFFT_OK) msg[j] = dbfft_last_error();
      }
    });
  }
  for (std::thread& x : th) x.join();
  for (int j = 0; j < nrhs; ++j)
    if (status[j] != DBFFT_OK) DB_THROW(status[j], "load " + std::to_string(j) + ": " + msg[j]);
  return DBFFT_OK;
  API_END
}

dbfft_status dbfft_set_lengths(dbfft_ctx* ctx, const double len[3]) {
  g_err.clear();
  API_BEGIN
  if (!ctx || !len) DB_THROW(DBFFT_EINVAL, "null argument");
  for (int a = 0; a < 3; ++a)
    if (!(len[a] > 0.0) || !std::isfinite(len[a])) DB_THROW(DBFFT_EINVAL, "cell lengths must be positive and finite");
  Ctx& c = *C(ctx);
  HIPCK(hipStreamSynchronize(c.st));
  c.g.il1 = 1.0 / len[0];
  c.g.il2 = 1.0 / len[1];
  c.g.il3 = 1.0 / len[2];
  // the captured PCG chunk holds the old geometry; the last solution refers to the old frequencies
  if (c.chunk_exec) HIPCK(hipGraphExecDestroy(c.chunk_exec));
  if (c.chunk_graph) HIPCK(hipGraphDestroy(c.chunk_graph));
  c.chunk_exec = nullptr;
  c.chunk_graph = nullptr;
  c.chunk_key.clear();
  c.solved = false;
  c.ck_n = 0;
  return DBFFT_OK;
  API_END
}

static double ratio_or_inf(double num, double den) {
  if (den == 0.0) return num == 0.0 ? 0.0 : INFINITY;
  return num / den;
}

dbfft_status dbfft_residuals(dbfft_ctx* ctx, const double* strain_dev, const double* stress_dev, const double load[9],
                             const uint8_t stress_mask[9], double out[4]) {
  g_err.clear();
  API_BEGIN
  if (!ctx || !out) DB_THROW(DBFFT_EINVAL, "null argument");
  Ctx& c = *C(ctx);
  if ((!strain_dev || !stress_dev) && !c.solved) DB_THROW(DBFFT_EINVAL, "no solution yet");
  const int nc = c.ncomp;
  const bool fin = c.kin == KIN_FINITE;
  double mt[9];
  for (int i = 0; i < 9; ++i) mt[i] = c.EU_st[i] + c.e_st[i];
  // equilibrium: the divergence coefficients of the stress field (the
  // residual of the Newton loop), whose weighted half-spectrum norm is the
  // mean square of div sigma over the voxels (Parseval); <sigma> from the DC bins
  const double* sig = stress_dev;
  if (!sig) {
    if (c.linear_material()) {
      set_macro(c, mt);
      strain_field(c, c.sol, c.mac_dev, c.fb, 1);
      sig = c.fb;
    } else {
      sig = c.fc;
    }
  }
  stress_residual(c, sig, c.t64, c.dc_dev);
  const double div2 = dot64(c, c.t64, c.t64);
  double sig_st[9], sig_rm[9] = {0};
  read_dc(c, sig_st);
  stored_to_rm(c.kin, sig_st, sig_rm);
  // compatibility: forward transform of the strain components, the curl
  // operator per frequency, back to real space, largest magnitude
  const double* eps = strain_dev;
  if (!eps) {
    set_macro(c, mt);
    strain_field(c, c.sol, c.mac_dev, c.fa);
    eps = c.fa;
  }
  Tables<double>& tb = c.td;
  const StridedGeom sx = xgeom(c), sy = ygeom(c);
  TangentArgs<double> tan = elastic_tangent<double>(c);
  launch_line<double>(LP_R2C, c.kin, eps, c.W, c.g, c.p3, tb.tw3, tb.rtw, tan, nullptr, nullptr, nullptr, nc, c.st,
                      nullptr, nullptr);
  launch_strided<double>(SP_PLAIN, c.W, c.W, nc, sy, c.g, c.p2, tb.tw2, -1, nullptr, c.st, nullptr);
  launch_strided<double>(SP_PLAIN, c.W, c.W, nc, sx, c.g, c.p1, tb.tw1, -1, nullptr, c.st, nullptr);
  for (int i = 0; i < nc; ++i)
    HIPCK(hipMemcpyAsync(c.red_host + i, static_cast<const double*>(c.W) + 2 * (size_t)i * c.g.nh, sizeof(double),
                         hipMemcpyDeviceToHost, c.st));
  launch_incompat(c.W, c.g, fin ? 1 : 0, c.st);
  launch_strided<double>(SP_PLAIN, c.W, c.W, nc, sx, c.g, c.p1, tb.tw1, +1, nullptr, c.st, nullptr);
  launch_strided<double>(SP_PLAIN, c.W, c.W, nc, sy, c.g, c.p2, tb.tw2, +1, nullptr, c.st, nullptr);
  launch_line<double>(LP_C2R, c.kin, c.W, c.fb, c.g, c.p3, tb.tw3, tb.rtw, tan, nullptr, nullptr, nullptr, nc, c.st,
                      nullptr, nullptr);
  HIPCK(hipGetLastError());
  HIPCK(hipStreamSynchronize(c.st));
  double eps_st[9] = {0}, eps_rm[9] = {0};
  for (int i = 0; i < nc; ++i) eps_st[i] = c.red_host[i];
  stored_to_rm(c.kin, eps_st, eps_rm);
  const double inc_max = max_abs_diff(c, c.fb, nullptr, (long long)nc * c.g.nvox);
  double sn = 0.0, en = 0.0;
  for (int i = 0; i < 9; ++i) {
    sn += sig_rm[i] * sig_rm[i];
    en += eps_rm[i] * eps_rm[i];
  }
  sn = std::sqrt(sn);
  en = std::sqrt(en);
  out[0] = ratio_or_inf(std::sqrt(std::max(div2, 0.0)), sn);
  out[1] = ratio_or_inf(inc_max, en);
  if (!load) {
    out[2] = out[3] = NAN;
  } else {
    double ne = 0.0, de = 0.0, ns = 0.0;
    bool anyE = false, anyS = false;
    for (int i = 0; i < 9; ++i) {
      const double id = (fin && i % 4 == 0) ? 1.0 : 0.0;
      if (stress_mask && stress_mask[i]) {
        anyS = true;
        ns += (sig_rm[i] - load[i]) * (sig_rm[i] - load[i]);
      } else {
        anyE = true;
        const double m = eps_rm[i] + id;
        ne += (m - load[i]) * (m - load[i]);
        de += (load[i] - id) * (load[i] - id);
      }
    }
    out[2] = anyE ? ratio_or_inf(std::sqrt(ne), std::sqrt(de)) : 0.0;
    out[3] = anyS ? ratio_or_inf(std::sqrt(ns), sn) : 0.0;
  }
  return DBFFT_OK;
  API_END
}

struct dbfft_batch {
  Batch impl;
};

dbfft_status dbfft_batch_create(dbfft_batch** out, dbfft_ctx* const* cells, int32_t ncell, int32_t use_graph) {
  g_err.clear();
  API_BEGIN
  if (!out || !cells || ncell < 1) DB_THROW(DBFFT_EINVAL, "null argument or empty batch");
  *out = nullptr;
  for (int r = 0; r < ncell; ++r)
    if (!cells[r]) DB_THROW(DBFFT_EINVAL, "null context in batch");
  Ctx& c0 = *C(cells[0]);
  for (int r = 1; r < ncell; ++r) {
    Ctx& c = *C(cells[r]);
    if (c.prec != c0.prec || c.kin != c0.kin || c.linear_material() != c0.linear_material() ||
        (!c0.linear_material() && c.mat != c0.mat))
      DB_THROW(DBFFT_EINVAL, "batched contexts need one precision, one kinematics and one material class");
  }
  dbfft_batch* h = new dbfft_batch();
  try {
    Batch& B = h->impl;
    for (int r = 0; r < ncell; ++r) {
      B.cells.push_back(C(cells[r]));
      B.handles.push_back(cells[r]);
    }
    B.prec = c0.prec;
    B.kin = c0.kin;
    B.ncomp = c0.ncomp;
    B.use_graph = use_graph != 0;
    for (int r = 0; r < ncell; ++r) HIPCK(hipStreamSynchronize(B.cells[r]->st));
    HIPCK(hipStreamCreateWithFlags(&B.st, hipStreamNonBlocking));
    if (B.prec == DBFFT_FP64) batch_build<double>(B);
    else batch_build<float>(B);
  } catch (...) {
    batch_release(&h->impl);
    delete h;
    throw;
  }
  *out = h;
  return DBFFT_OK;
  API_END
}

// Small-strain cells of 96^3 voxels and more are solved cell by cell with
// the single-cell passes, whose launches already have a thousand or more
// blocks there (measured faster than the batched passes from 96^3 up).
static bool solve_cellwise(const Batch& B) {
  for (const Ctx* c : B.cells)
    if (!(c->kin == KIN_SMALL && c->g.nvox >= 96LL * 96 * 96)) return false;
  return true;
}

constexpr int kCellLanes = 2;  // cells solved at once by the cell-by-cell path

// dbfft_solve on every cell, kCellLanes cells at a time: each lane is a
// host thread (the calling one for the first lane) and a non-blocking
// stream of the batch, on which the cell's context enqueues for the call
// (its own stream is synchronized first and given back afterwards).  Two solves at once fill each other's launch
// gaps.  A context listed twice keeps every solve in one lane.  Returns the
// worst status as dbfft_batch_solve does.
static dbfft_status batch_solve_cellwise(Batch& B, const double* loads, const uint8_t* masks, int ninc, double dt,
                                         const dbfft_opts& o, dbfft_info* infos) {
  const int n = (int)B.cells.size();
  bool dup = false;
  for (int a = 0; a < n && !dup; ++a)
    for (int b = a + 1; b < n; ++b)
      if (B.cells[a] == B.cells[b]) dup = true;
  const int nl = dup ? 1 : std::min(kCellLanes, n);
  while ((int)B.lane_st.size() < nl) {
    hipStream_t s = nullptr;
    HIPCK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    B.lane_st.push_back(s);
  }
  std::vector<int> status(n, DBFFT_OK);
  std::vector<std::string> msg(n);
  auto lane = [&](int t) {
    for (int r = t; r < n; r += nl) {
      Ctx& c = *B.cells[r];
      if ((t > 0 && hipSetDevice(c.dev) != hipSuccess) || hipStreamSynchronize(c.st) != hipSuccess) {
        status[r] = DBFFT_EHIP;
        msg[r] = "cannot select the cell's device or synchronize its stream";
        continue;
      }
      const hipStream_t own = c.st;
      c.st = B.lane_st[t];
      status[r] = dbfft_solve(B.handles[r], loads + 9 * (size_t)r, masks + 9 * (size_t)r, ninc, dt, &o, &infos[r]);
      if (status[r] != DBFFT_OK) msg[r] = dbfft_last_error();
      (void)hipStreamSynchronize(c.st);
      c.st = own;
    }
  };
  std::vector<std::thread> th;
  for (int t = 1; t < nl; ++t) th.emplace_back(lane, t);
  lane(0);
  for (std::thread& x : th) x.join();
  int worst = DBFFT_OK;
  for (int r = 0; r < n; ++r) {
    if (status[r] == DBFFT_OK) continue;
    if (status[r] != DBFFT_ENOTCONV && status[r] != DBFFT_EBREAKDOWN)
      DB_THROW(status[r], "cell " + std::to_string(r) + ": " + msg[r]);
    worst = status[r];
    g_err = "cell " + std::to_string(r) + ": " + msg[r];
  }
  return (dbfft_status)worst;
}

dbfft_status dbfft_batch_solve(dbfft_batch* b, const double* loads, const uint8_t* stress_masks, int32_t n_increments,
                               double dt, const dbfft_opts* opts, dbfft_info* infos) {
  g_err.clear();
  API_BEGIN
  if (!b || !loads || !stress_masks || !infos) DB_THROW(DBFFT_EINVAL, "null argument");
  Batch& B = b->impl;
  const int n = (int)B.cells.size();
  dbfft_opts o;
  if (opts) o = *opts;
  else dbfft_default_opts(&o);
  o.checkpoint = 0;  // batches keep no checkpoints
  if (o.coarse_kc != 0) DB_THROW(DBFFT_EUNSUPPORTED, "opts.coarse_kc applies to dbfft_solve_block");
  for (int r = 0; r < n; ++r) {
    const Ctx& c = *B.cells[r];
    if (c.kin == KIN_SMALL)
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
          if ((stress_masks[9 * r + i * 3 + j] != 0) != (stress_masks[9 * r + j * 3 + i] != 0))
            DB_THROW(DBFFT_EINVAL, "small strains need a symmetric stress mask");
          if (loads[9 * r + i * 3 + j] != loads[9 * r + j * 3 + i]) DB_THROW(DBFFT_EINVAL, "small strains need a symmetric load");
        }
  }
  if (!B.cells[0]->linear_material()) {
    if (n_increments < 1) DB_THROW(DBFFT_EINVAL, "n_increments must be >= 1");
    if (B.cells[0]->mat == DBFFT_MAT_J2VP_CUBIC && !(dt > 0.0)) DB_THROW(DBFFT_EINVAL, "dt must be > 0");
  }
  if (solve_cellwise(B)) return batch_solve_cellwise(B, loads, stress_masks, n_increments, dt, o, infos);
  std::vector<int> st = (B.prec == DBFFT_FP64) ? batch_solve_t<double>(B, loads, stress_masks, n_increments, dt, o, infos)
                                               : batch_solve_t<float>(B, loads, stress_masks, n_increments, dt, o, infos);
  int worst = DBFFT_OK;
  for (int v : st)
    if (v != DBFFT_OK) worst = v;
  if (worst != DBFFT_OK && g_err.empty()) g_err = "at least one cell of the batch did not converge";
  return (dbfft_status)worst;
  API_END
}

dbfft_status dbfft_batch_tiles(dbfft_batch* b, int32_t* tiles) {
  g_err.clear();
  API_BEGIN
  if (!b || !tiles) DB_THROW(DBFFT_EINVAL, "null argument");
  Batch& B = b->impl;
  for (size_t r = 0; r < B.cells.size(); ++r) {
    tiles[3 * r] = B.tzx[r];
    tiles[3 * r + 1] = B.tzy[r];
    tiles[3 * r + 2] = B.L[r];
  }
  return DBFFT_OK;
  API_END
}

void dbfft_batch_destroy(dbfft_batch* b) {
  if (!b) return;
  batch_release(&b->impl);
  delete b;
}

dbfft_status dbfft_get_solution(dbfft_ctx* ctx, void* a_dev, double e_macro[9]) {
  g_err.clear();
  API_BEGIN
  if (!ctx) DB_THROW(DBFFT_EINVAL, "null context");
  Ctx& c = *C(ctx);
  if (!c.solved) DB_THROW(DBFFT_EINVAL, "no solution yet");
  if (a_dev)
    HIPCK(hipMemcpyAsync(a_dev, c.sol, 3 * (size_t)c.g.nh * 2 * sizeof(double), hipMemcpyDeviceToDevice, c.st));
  if (e_macro) stored_to_rm(c.kin, c.e_st, e_macro);
  HIPCK(hipStreamSynchronize(c.st));
  return DBFFT_OK;
  API_END
}

// J2 adjoint through the checkpointed increments of the last solve (the
// recursion is stated with dbfft_adjoint in the header)
static void j2_adjoint(Ctx& c, const double G[9], const double H[9], double* grad_dev) {
  bool all_stress = true;
  for (int i = 0; i < 9; ++i) all_stress = all_stress && c.last_mask[i];
  if (all_stress) DB_THROW(DBFFT_EUNSUPPORTED, "J2 adjoint with every component stress-controlled");
  if (c.ck_n <= 0)
    DB_THROW(DBFFT_EINVAL, "the J2 adjoint needs the checkpoints of the last solve (opts.checkpoint = 1)");
  const long long N = c.g.nvox;
  const size_t vs = 6 * (size_t)c.g.nh;
  if (!c.adj_lam) c.adj_lam = static_cast<double*>(dalloc(6 * (size_t)N * sizeof(double)));
  HIPCK(hipMemsetAsync(c.adj_lam, 0, 6 * (size_t)N * sizeof(double), c.st));
  HIPCK(hipMemsetAsync(grad_dev, 0, (size_t)N * sizeof(double), c.st));
  dbfft_opts o;
  dbfft_default_opts(&o);
  o.tol = 1e-12;
  o.tol_load = 1e-12;
  const MacroSet ms = macro_set(c, c.last_mask);
  // converged strain of increment n and the plastic strain it started from;
  // the return map there gives K_n (tanf), p_n (state_new) and sigma_n (fc)
  auto restore = [&](int n) {
    const double* ck = c.ck_buf + (size_t)n * ck_stride(c);
    set_macro(c, c.ck_mt[n].data());
    strain_field(c, ck, c.mac_dev, c.fa);
    HIPCK(hipMemcpyAsync(c.state, ck + vs, 6 * (size_t)N * sizeof(double), hipMemcpyDeviceToDevice, c.st));
    material_update(c, c.fa, c.fc, c.ck_dt);
  };
  for (int n = c.ck_n - 1; n >= 0; --n) {
    restore(n);
    const bool last = n == c.ck_n - 1;
    double Urm[9] = {0}, Lrm[9] = {0};
    if (last)
      for (int i = 0; i < 9; ++i) {
        Urm[i] = c.last_mask[i] ? 0.0 : G[i];
        Lrm[i] = c.last_mask[i] ? -H[i] : G[i];
      }
    double EU2[9], lst[9];
    rm_to_stored(c.kin, Urm, EU2);
    rm_to_stored(c.kin, Lrm, lst);
    double sbar[kMaxMacro] = {0};
    for (int a = 0; a < ms.nS; ++a) sbar[a] = bdot(c.kin, ms.bst[a], lst);
    // residual of the affine stress law K_n : eps + A_n at eps = EU
    launch_j2_adj_prestress(c.adj_lam, c.tanf, c.grain, c.grainS, EU2, N, c.fc, c.st);
    stress_residual(c, c.fc, c.b, c.dc_dev);
    double dc0[9];
    read_dc(c, dc0);
    double re0[kMaxMacro] = {0}, r2 = std::max(dot64(c, c.b, c.b), 0.0);
    for (int a = 0; a < ms.nS; ++a) {
      re0[a] = sbar[a] - bdot(c.kin, ms.bst[a], dc0);
      r2 += re0[a] * re0[a];
    }
    // the residual test is relative to the initial residual: the mean
    // stress of these problems changes sign along the path
    LinOut lo = r2 > 0.0 ? linear_solve_b(c, ms, dc0, re0, o, c.sol2, std::sqrt(r2)) : LinOut{};
    if (!(r2 > 0.0)) HIPCK(hipMemsetAsync(c.sol2, 0, 6 * (size_t)c.g.nh * sizeof(double), c.st));
    if (lo.status != DBFFT_OK) DB_THROW(lo.status, "adjoint solve did not converge");
    double mt2[9];
    for (int i = 0; i < 9; ++i) mt2[i] = EU2[i];
    for (int a = 0; a < ms.nS; ++a)
      for (int i = 0; i < 9; ++i) mt2[i] += lo.e_coef[a] * ms.bst[a][i];
    set_macro(c, mt2);
    strain_field(c, c.sol2, c.mac_dev, c.fb);
    launch_j2_adj_back(c.adj_lam, c.tanf, c.grain, c.grainS, c.fb, c.state_new, c.state, -c.j2_m / (double)N, N,
                       grad_dev, c.st);
  }
  // the state, tangent and fields as the solve left them
  restore(c.ck_n - 1);
  std::swap(c.state, c.state_new);
}

dbfft_status dbfft_adjoint(dbfft_ctx* ctx, const double G[9], const double H[9], double* grad_dev, double* J_out) {
  g_err.clear();
  API_BEGIN
  if (!ctx || !G || !H || !grad_dev) DB_THROW(DBFFT_EINVAL, "null argument");
  Ctx& c = *C(ctx);
  const bool hyper = (c.mat == DBFFT_MAT_NEOHOOKE || c.mat == DBFFT_MAT_SVK) && c.kin == KIN_FINITE;
  const bool j2 = c.mat == DBFFT_MAT_J2VP_CUBIC && c.kin == KIN_SMALL;
  if (!hyper && !j2 && (c.mat != DBFFT_MAT_ISO_FIELD || c.kin != KIN_SMALL))
    DB_THROW(DBFFT_EUNSUPPORTED,
             "the adjoint handles ISO_FIELD and J2VP_CUBIC materials under small strains and NEOHOOKE / SVK under "
             "finite strains");
  if (!c.solved) DB_THROW(DBFFT_EINVAL, "no forward solution");
  if (!hyper)
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j)
        if (G[i * 3 + j] != G[j * 3 + i] || H[i * 3 + j] != H[j * 3 + i])
          DB_THROW(DBFFT_EINVAL, "G and H must be symmetric");
  if (!c.sol2) c.sol2 = static_cast<double*>(dalloc(3 * (size_t)c.g.nh * 2 * sizeof(double)));
  auto objective = [&]() {
    double J = 0.0;
    for (int i = 0; i < 9; ++i) J += G[i] * c.sig_rm[i] + H[i] * c.eps_rm[i];
    return J;
  };
  if (j2) {
    j2_adjoint(c, G, H, grad_dev);
    HIPCK(hipGetLastError());
    HIPCK(hipStreamSynchronize(c.st));
    if (J_out) *J_out = objective();
    return DBFFT_OK;
  }
  dbfft_opts o;
  dbfft_default_opts(&o);
  o.tol = 1e-12;
  o.tol_load = 1e-12;
  if (hyper) {
    // the final state's nominal stress and tangent (hyperelastic: the
    // response at the end of the path depends on that state only)
    double mt[9];
    for (int i = 0; i < 9; ++i) mt[i] = c.EU_st[i] + c.e_st[i];
    set_macro(c, mt);
    strain_field(c, c.sol, c.mac_dev, c.fa);
    material_update(c, c.fa, c.fc, 1.0);
  }
  const MacroSet ms = macro_set(c, c.last_mask);
  double Urm[9], Lrm[9];
  for (int i = 0; i < 9; ++i) {
    Urm[i] = c.last_mask[i] ? 0.0 : G[i];
    Lrm[i] = c.last_mask[i] ? -H[i] : G[i];
  }
  double EU2[9], lst[9];
  rm_to_stored(c.kin, Urm, EU2);
  rm_to_stored(c.kin, Lrm, lst);
  double sbar[kMaxMacro] = {0};
  for (int a = 0; a < ms.nS; ++a) sbar[a] = bdot(c.kin, ms.bst[a], lst);
  LinOut lo = linear_solve(c, EU2, ms, sbar, o, c.sol2);
  if (lo.status != DBFFT_OK) DB_THROW(lo.status, "adjoint solve did not converge");
  double mt2[9];
  for (int i = 0; i < 9; ++i) mt2[i] = EU2[i];
  for (int a = 0; a < ms.nS; ++a)
    for (int i = 0; i < 9; ++i) mt2[i] += lo.e_coef[a] * ms.bst[a][i];
  if (hyper) {
    // P is linear in the law's moduli: dP/dtheta = P at theta = 1
    set_macro(c, mt2);
    strain_field(c, c.sol2, c.mac_dev, c.fb);
    launch_contract(c.fb, c.fc, 9, c.g.nvox, grad_dev, c.g.inv_nvox, c.st);
  } else {
    double mt[9];
    for (int i = 0; i < 9; ++i) mt[i] = c.EU_st[i] + c.e_st[i];
    set_macro(c, mt);
    strain_field(c, c.sol, c.mac_dev, c.fa);
    set_macro(c, mt2);
    strain_field(c, c.sol2, c.mac_dev, c.fb);
    launch_adjoint_density(c.fa, c.fb, c.lam1, c.mu1, c.g.nvox, grad_dev, c.g.inv_nvox, c.st);
  }
  HIPCK(hipGetLastError());
  HIPCK(hipStreamSynchronize(c.st));
  if (J_out) *J_out = objective();
  return DBFFT_OK;
  API_END
}

}  // extern "C"
