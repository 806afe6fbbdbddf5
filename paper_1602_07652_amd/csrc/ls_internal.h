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

typedef double2 cplx;

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
  cplx* fac;         // block-cyclic-reduction factors (offsets in levels)
  size_t fac_elems;
  std::vector<SlabLevel> levels;  // levels[0] .. levels[nlev-1]; last has nl == 1
  cplx* g;           // right-hand side g^l kept across the two sweeps [n][q]
  cplx* w;           // downward-sweep solution w^l [n][q]
};

// Contiguous set of grid vectors used as a Krylov basis.
struct KrylovSpace {
  cplx* base = nullptr;
  int cap = 0;
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
  cplx* vtmp = nullptr;          // grid vectors for Alg. 2 [3][n*n]

  // Krylov workspace (grid vectors), grown on demand
  KrylovSpace innerV, innerZ, outerV, outerZ;
  cplx* inner_rhs = nullptr;     // A r of the inner level
  cplx* red = nullptr;           // reduction partials
  cplx* dotbuf = nullptr;        // device results of multi-dots
  std::vector<void*> allocs;     // every device allocation, freed at destroy
};

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
ls_status apply_H(ls_plan* p, const cplx* v, cplx* y, int batch, double sign_identity, double scale_conv);
// stencil.hip
ls_status stencils_build(ls_plan* p, const cplx* circ);
ls_status stencil_apply_A(ls_plan* p, const cplx* r, cplx* y, int batch);
ls_status stencil_apply_C(ls_plan* p, const cplx* v, cplx* y, int batch);
ls_status stencil_residual_C(ls_plan* p, const cplx* g, const cplx* u, cplx* e);  // e = g - C u
// slab.hip
ls_status slabs_build(ls_plan* p);
ls_status slab_solve_frame(ls_plan* p, Slab& s, cplx* x);        // in place on x [n][q]
ls_status sweep_apply(ls_plan* p, int orient, const cplx* g, cplx* v, bool accumulate);
ls_status bidirectional_apply(ls_plan* p, const cplx* g, cplx* v);
// blas.hip
ls_status vec_multidot(ls_plan* p, const cplx* V, int k, size_t stride, const cplx* w, size_t N, cplx* out_host);
ls_status vec_multiaxpy(ls_plan* p, cplx* w, const cplx* V, int k, size_t stride, const cplx* coef_host, size_t N);
ls_status vec_norm(ls_plan* p, const cplx* w, size_t N, double* out_host);
ls_status vec_scale_copy(ls_plan* p, cplx* y, const cplx* x, double s, size_t N);
ls_status vec_lincomb(ls_plan* p, cplx* x, const cplx* Z, int k, size_t stride, const cplx* coef_host, size_t N);
ls_status vec_axpy(ls_plan* p, cplx* y, const cplx* x, cplx a, size_t N);  // y += a x
ls_status vec_zero(ls_plan* p, cplx* y, size_t N);
ls_status vec_copy(ls_plan* p, cplx* y, const cplx* x, size_t N);
