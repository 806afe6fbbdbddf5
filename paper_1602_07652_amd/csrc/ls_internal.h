// Internal declarations of the MI355X Lippmann-Schwinger library.
// Everything here is private to the shared library; the public ABI is
// include/ls.h.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/ls.h"
#include "../../include/ls_fno.h"

typedef double2 cplx;
typedef float2 fcplx;

// ---------------------------------------------------------------- errors
void ls_set_error(const std::string& msg);

#define LS_HIP(call)                                                               \
  do {                                                                             \
    hipError_t e_ = (call);                                                        \
    if (e_ != hipSuccess) {                                                        \
      ls_set_error(std::string(#call) + ": " + hipGetErrorString(e_));              \
      return LS_EDEVICE;                                                           \
    }                                                                              \
  } while (0)

#define LS_TRY(expr)                \
  do {                                \
    ls_status s_ = (expr);            \
    if (s_ != LS_OK) return s_;       \
  } while (0)

// ------------------------------------------------------- complex helpers
__host__ __device__ __forceinline__ cplx cmk(double re, double im) { return make_double2(re, im); }
__host__ __device__ __forceinline__ cplx cadd(cplx a, cplx b) { return cmk(a.x + b.x, a.y + b.y); }
__host__ __device__ __forceinline__ cplx csub(cplx a, cplx b) { return cmk(a.x - b.x, a.y - b.y); }
__host__ __device__ __forceinline__ cplx cmul(cplx a, cplx b) {
  return cmk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__host__ __device__ __forceinline__ cplx cconj(cplx a) { return cmk(a.x, -a.y); }
__host__ __device__ __forceinline__ cplx cscale(cplx a, double s) { return cmk(a.x * s, a.y * s); }
// acc + a*b
__host__ __device__ __forceinline__ cplx cfma(cplx a, cplx b, cplx acc) {
  return cmk(fma(a.x, b.x, fma(-a.y, b.y, acc.x)), fma(a.x, b.y, fma(a.y, b.x, acc.y)));
}
// acc + conj(a)*b
__host__ __device__ __forceinline__ cplx cfmaconj(cplx a, cplx b, cplx acc) {
  return cmk(fma(a.x, b.x, fma(a.y, b.y, acc.x)), fma(a.x, b.y, fma(-a.y, b.x, acc.y)));
}

// Precision-generic complex helpers (C = double2 or float2; arithmetic in
// the precision of C).
template <typename C>
__host__ __device__ __forceinline__ C tmk(double re, double im) {
  C r;
  r.x = re;
  r.y = im;
  return r;
}
template <typename C>
__host__ __device__ __forceinline__ C tadd(C a, C b) { C r; r.x = a.x + b.x; r.y = a.y + b.y; return r; }
template <typename C>
__host__ __device__ __forceinline__ C tsub(C a, C b) { C r; r.x = a.x - b.x; r.y = a.y - b.y; return r; }
template <typename C>
__host__ __device__ __forceinline__ C tmul(C a, C b) {
  C r;
  r.x = a.x * b.x - a.y * b.y;
  r.y = a.x * b.y + a.y * b.x;
  return r;
}
template <typename C>
__host__ __device__ __forceinline__ C tfma(C a, C b, C acc) {  // acc + a*b
  C r;
  r.x = fma(a.x, b.x, fma(-a.y, b.y, acc.x));
  r.y = fma(a.x, b.y, fma(a.y, b.x, acc.y));
  return r;
}
template <typename C>
__host__ __device__ __forceinline__ C tneg(C a) { C r; r.x = -a.x; r.y = -a.y; return r; }

// ---------------------------------------------------------------- slabs
// One extended layer in its own frame: long axis index i in [0, n) (x for
// horizontal layers, z for vertical ones), short axis index r in [0, q)
// for the line z0 + r (z for horizontal, x for vertical).
struct SlabLevel {
  int nl;            // blocks at this level
  size_t off_dinv;   // odd blocks: Dinv            [nl/2][q][q] (column-major blocks)
  size_t off_dinvl;  // odd blocks: Dinv * L        (levels >= 1)
  size_t off_dinvu;  // odd blocks: Dinv * U        (levels >= 1)
  size_t off_pm;     // even blocks: L * Dinv(k-1)  (levels >= 1)
  size_t off_pp;     // even blocks: U * Dinv(k+1)  (levels >= 1)
};

struct Slab {
  int orient;        // 0 horizontal, 1 vertical
  int idx;           // layer index l
  int a, b, z0, z1;  // layer lines and extended lines (short axis)
  int q;             // z1 - z0 + 1
  cplx* coef;        // [n][q][9] assembled local matrix C^l (stencil form)
  // level-0 couplings of each block to its neighbours, [n][6][q] (row r of
  // block k: c = 2 (dZ + 1) + side, the coefficient of row r + dZ of block
  // k - 1 (side 0) or k + 1 (side 1)), in the plan's precision
  cplx* cpl = nullptr;
  fcplx* cpl32 = nullptr;
  // level-0 odd blocks as tridiagonal systems [n/2][3][q]: the sub-diagonal,
  // diagonal and super-diagonal of each block, in the plan's precision
  cplx* tri = nullptr;
  fcplx* tri32 = nullptr;
  cplx* fac;         // block-cyclic-reduction factors (offsets in levels)
  size_t fac_elems;
  std::vector<SlabLevel> levels;  // levels[0] .. levels[nlev-1]; last has nl == 1
  cplx* g;           // right-hand side g^l kept across the two sweeps [n][q]
  cplx* w;           // downward-sweep solution w^l [n][q]
  // FP32 plans: FP32 copies used by the solves (factors computed in FP64)
  fcplx* coef32;
  fcplx* fac32;
  fcplx* g32;
  fcplx* w32;
  // Top of the reduction as one dense operator: the levels from top_level
  // up (top_level >= 1, at most 16 blocks there, 8 on plans with the
  // decoupled sweep and few right-hand sides) solved by y = top t on the
  // top_n = nl * q unknowns of that level; row-major [top_n][top_n].
  // top_level = -1: no such operator (the chain runs every level).
  int top_level;
  int top_n;
  cplx* top;
  fcplx* top32;
  fcplx* top32T;  // FP32 plans with max_batch >= 16: column-major copy [top_n][top_n]
  // Trace-transfer maps of the decoupled sweep (opt.sweep == LS_SWEEP_DECOUPLED),
  // row-major [2n][2n] in the plan's precision (null where the slab needs none):
  // mT = R_tau (C^l)^{-1} E, mU = R_sigma (C^l)^{-1} E, mV = R_sigma (C^l)^{-1} F
  // (E, F: the downward and upward trace-source injections of the layer,
  // R_tau, R_sigma: the two grid lines its neighbours read).
  cplx* mT;
  cplx* mU;
  cplx* mV;
  fcplx* mT32;
  fcplx* mU32;
  fcplx* mV32;
};

// Contiguous set of grid vectors used as a Krylov basis.
template <typename T>
struct KrylovSpaceT {
  T* base = nullptr;
  int cap = 0;
};
typedef KrylovSpaceT<cplx> KrylovSpace;

// Device state of the FP32 operator (refinement path).
struct Fp32State {
  float* m = nullptr;
  fcplx* spec = nullptr;
  fcplx* tw = nullptr;
  fcplx* fft_work = nullptr;
  fcplx* stencil = nullptr;   // alpha, beta, alphaT, betaT as float2
};

// Real type of a complex type.
template <typename T>
struct CT;
template <>
struct CT<cplx> { typedef double R; };
template <>
struct CT<fcplx> { typedef float R; };

// Everything the FFT convolution needs, for one precision.
template <typename T, typename R>
struct ApplyView {
  const R* m;
  const T* spec;
  const T* tw;
  T* work;
  int n, ss;
  hipStream_t stream;
  int col_variant;  // column-pass tile variant chosen by the autotuner
  int cus;          // compute units of the device (persistent grids)
};

// A captured inner-preconditioner application.
struct GraphEntry {
  const void* in;
  void* out;
  int B;
  int elem;  // sizeof the complex type
  hipGraphExec_t exec;
};

// ---------------------------------------------------------------- plan
struct ls_plan {
  int n = 0, P = 0, logP = 0, L = 0, spec_side = 0;
  double h = 0, omega = 0;
  ls_options opt{};
  hipStream_t stream = nullptr;
  int device = 0;

  double* m = nullptr;      // [n*n]
  cplx* spec = nullptr;     // quarter spectrum [spec_side][spec_side], scaled by omega^2/P^2
  cplx* tw = nullptr;       // twiddles exp(-2 pi i k / P), k < P
  cplx* fft_work = nullptr; // [max_batch][n*P] intermediate of ls_apply

  cplx alpha_h[81], beta_h[81];  // stencil tables (host copy)
  cplx* stencil_d = nullptr;     // device: alpha[81], beta[81], alphaT[81], betaT[81]

  std::vector<Slab> slabs[2];
  cplx* slab_work = nullptr;     // [n][qmax] scratch for one slab solve
  cplx* slab_work2 = nullptr;    // second scratch
  cplx* slab_elim = nullptr;     // [n][qmax] eliminated right-hand sides of one solve
  cplx* vtmp = nullptr;          // grid vectors for Alg. 2 [3][n*n]
  fcplx* slab_work32 = nullptr;  // FP32 plans: the two slab scratch vectors
  fcplx* slab_work32b = nullptr;
  fcplx* slab_elim32 = nullptr;
  fcplx* top_part32 = nullptr;   // batched top operator: per-slice partial products
  fcplx* vtmp32 = nullptr;       // FP32 plans: grid vectors [3][n*n]
  cplx* traces = nullptr;        // decoupled sweep: tau and sigma traces [2][L][2n]
  fcplx* traces32 = nullptr;

  // Krylov workspace (grid vectors), grown on demand
  KrylovSpace innerV, innerZ, outerV, outerZ;
  cplx* inner_rhs = nullptr;     // A r of the inner level
  KrylovSpaceT<fcplx> innerV32, innerZ32, outerV32, outerZ32;
  fcplx* inner_rhs32 = nullptr;
  cplx* red = nullptr;           // reduction partials
  cplx* dotbuf = nullptr;        // device results of multi-dots / update coefficients
  cplx* hres = nullptr;          // pinned host twins of dotbuf: results, coefficients
  cplx* hcoef = nullptr;
  hipEvent_t coef_ev = nullptr;  // recorded after the last coefficient upload
  bool coef_pending = false;
  std::vector<void*> allocs;     // every device allocation, freed at destroy

  bool fp32 = false;             // FP32 operator + FP64 refinement
  Fp32State f32;

  bool own_stream = false;       // created by the plan (caller passed NULL)
  std::vector<GraphEntry> graphs;
  cplx* solve_buf = nullptr;     // FP64 plans, learned solves: two grid-vector batches
  int col_variant64 = 0, col_variant32 = 0;  // autotuned FFT column-pass variants
  float tune_ms64[8] = {}, tune_ms32[8] = {};  // one per FFT column-pass variant
  int cus = 256;                 // compute units of the plan's device
  // wall time of the off-line stages (ls_plan_timings): kernel samples and
  // circulant, stencils, spectrum, slab assembly, slab factorisation, top
  // operators, trace-transfer maps, FFT autotuning, whole ls_plan_create
  double stage_ms[9] = {};
  // decoupled sweep: the layers of each orientation grouped by slab shape
  // (same q and level structure: one multi-slab launch per level step and
  // group), every layer's elimination scratch [L][n][set_qmax] in the
  // plan's precision, and side streams (with fork / join events) that run
  // the groups after the first concurrently
  std::vector<std::vector<int>> dec_groups[2];
  void* set_elim = nullptr;
  // the one-right-hand-side slab solves take their level-0 odd steps as
  // tridiagonal solves (every block's agreed with its dense inverse at plan
  // creation)
  bool tri_ok = false;
  int set_qmax = 0;
  static constexpr int kSide = 4;
  hipStream_t side[kSide] = {};
  hipEvent_t side_fork = nullptr;
  hipEvent_t side_join[kSide] = {};
};

inline ApplyView<cplx, double> view64(ls_plan* p) {
  return ApplyView<cplx, double>{p->m,    p->spec,       p->tw,     p->fft_work,
                                 p->n,    p->spec_side,  p->stream, p->col_variant64, p->cus};
}
inline ApplyView<fcplx, float> view32(ls_plan* p) {
  return ApplyView<fcplx, float>{p->f32.m, p->f32.spec,   p->f32.tw, p->f32.fft_work,
                                 p->n,     p->spec_side,  p->stream, p->col_variant32, p->cus};
}

// fno.hip: the network as a residual map z = r + s y(m, u_I, r / s) on the
// handle's stream; the stream can be swapped for the duration of a solve.
template <typename T>
ls_status fno_residual_map(ls_fno* f, int n, int S, const double* m, size_t mstr, const double* uI,
                           const T* r, T* z);
hipStream_t fno_swap_stream(ls_fno* f, hipStream_t s);
int fno_max_batch(const ls_fno* f);
int fno_max_n(const ls_fno* f);

// host wall clock in ms after the plan's stream has drained (stage timers)
double plan_clock_ms(ls_plan* p);
// device memory helpers (record in plan->allocs)
ls_status plan_alloc(ls_plan* p, void** ptr, size_t bytes);

// -------------------------------------------------------- module entry points
// hankel.hip
ls_status launch_circulant(ls_plan* p, cplx* c);                 // P x P circulant of w
ls_status launch_kernel_samples(ls_plan* p, cplx* w);            // (2n-1)^2 samples
// fft.hip
ls_status fft_setup_twiddles(ls_plan* p);
ls_status fft2_full_forward(ls_plan* p, cplx* c);                // in place, P x P row-major
ls_status spectrum_extract(ls_plan* p, const cplx* c);           // -> p->spec
ls_status spectrum_to_f32(ls_plan* p);                            // p->f32.spec from p->spec
ls_status apply_H(ls_plan* p, const cplx* v, cplx* y, int batch, double sign_identity, double scale_conv);
ls_status apply_H32(ls_plan* p, const fcplx* v, fcplx* y, int batch, double sign_identity, double scale_conv);
constexpr int kFftVariants = 8;  // FFT column-pass variants (fft.hip)
ls_status fft_autotune(ls_plan* p);
// stencil.hip
ls_status stencils_build(ls_plan* p, const cplx* circ);
ls_status stencil_apply_A(ls_plan* p, const cplx* r, cplx* y, int batch);
ls_status stencil_apply_C(ls_plan* p, const cplx* v, cplx* y, int batch);
ls_status stencil_residual_C(ls_plan* p, const cplx* g, const cplx* u, cplx* e, int batch = 1);  // e = g - C u
ls_status stencil_apply_A(ls_plan* p, const fcplx* r, fcplx* y, int batch);
ls_status stencil_apply_C(ls_plan* p, const fcplx* v, fcplx* y, int batch);
ls_status stencil_residual_C(ls_plan* p, const fcplx* g, const fcplx* u, fcplx* e, int batch = 1);
ls_status stencils_to_f32(ls_plan* p);
// slab.hip
ls_status slabs_build(ls_plan* p);
// y = C_slab^{-1} g for B right-hand sides [B][n][q] in the slab frame;
// g is not modified and must not alias y
ls_status slab_solve(ls_plan* p, Slab& s, const cplx* g, cplx* y, int B);
ls_status slab_solve(ls_plan* p, Slab& s, const fcplx* g, fcplx* y, int B);
// B right-hand sides [B][n][n] at once
ls_status sweep_apply(ls_plan* p, int orient, const cplx* g, cplx* v, bool accumulate, int B = 1);
ls_status sweep_apply(ls_plan* p, int orient, const fcplx* g, fcplx* v, bool accumulate, int B = 1);
ls_status bidirectional_apply(ls_plan* p, const cplx* g, cplx* v, int B = 1);
ls_status bidirectional_apply(ls_plan* p, const fcplx* g, fcplx* v, int B = 1);
// allocation-free single-right-hand-side slab solve (scratch in a static
// device array, set up once per device by static_scratch_init)
ls_status static_scratch_init(int device);
size_t static_scratch_bytes();
ls_status slab_solve_noalloc(ls_plan* p, Slab& s, const cplx* b, cplx* x);
// blas.hip (each for T = cplx and T = fcplx; inner products in FP64)
// Batched forms act on B right-hand sides stored [B][N] (vector i of a
// Krylov set at V + i*stride, stride >= B*N); coefficient arrays are [B][k].
#define LS_BLAS_DECLS(T)                                                                           \
  ls_status vec_multidot(ls_plan* p, const T* V, int k, size_t stride, const T* w, size_t N,      \
                         int B, cplx* out_host);                                                   \
  ls_status vec_multiaxpy(ls_plan* p, T* w, const T* V, int k, size_t stride,                     \
                          const cplx* coef_host, size_t N, int B);                                 \
  ls_status vec_lincomb(ls_plan* p, T* x, const T* Z, int k, size_t stride,                       \
                        const cplx* coef_host, size_t N, int B);                                   \
  ls_status vec_norms(ls_plan* p, const T* w, size_t N, int B, double* out_host);                 \
  /* classical Gram-Schmidt with one re-orthogonalisation, 1 <= k <= 8 */                         \
  ls_status vec_cgs2(ls_plan* p, const T* V, int k, size_t stride, T* w, size_t N, int B,         \
                     cplx* h1_host, cplx* h2_host, double* nrm2_host);                             \
  /* z = alpha zt with alpha = (w^H g) / (w^H w) per right-hand side, on the */                    \
  /* device (no host transfer): one step of right-preconditioned GMRES */                        \
  ls_status vec_minres_scale(ls_plan* p, const T* w, const T* g, const T* zt, T* z, size_t N,      \
                             int B);                                                               \
  ls_status vec_norm(ls_plan* p, const T* w, size_t N, double* out_host);                         \
  ls_status vec_scale_b(ls_plan* p, T* y, const T* x, const double* s_host, size_t N, int B);     \
  ls_status vec_scale_copy(ls_plan* p, T* y, const T* x, double s, size_t N);                     \
  ls_status vec_axpy(ls_plan* p, T* y, const T* x, cplx a, size_t N);                            \
  ls_status vec_zero(ls_plan* p, T* y, size_t N);                                                 \
  ls_status vec_copy(ls_plan* p, T* y, const T* x, size_t N);
LS_BLAS_DECLS(cplx)
LS_BLAS_DECLS(fcplx)
ls_status vec_to_f32(ls_plan* p, fcplx* y, const cplx* x, double s, size_t N);          // y = s x
ls_status vec_to_f32_b(ls_plan* p, fcplx* y, const cplx* x, const double* s_host, size_t N, int B);
ls_status vec_from_f32_b(ls_plan* p, cplx* y, const cplx* y0, const fcplx* x, const double* s_host,
                         size_t N, int B);
ls_status vec_from_f32(ls_plan* p, cplx* y, const cplx* y0, const fcplx* x, double s,  // y = y0 + s x
                       size_t N);
