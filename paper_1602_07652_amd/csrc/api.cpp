// C ABI of the library (include/ls.h): plan construction (the off-line
// stage of Section 4.1), the operators, and the two GMRES levels of
// Section 4 (Alg. 3 inside, flexible GMRES outside) driven from the host
// with all vectors on the device.
//
// Krylov method (both levels): x0 = 0; classical Gram-Schmidt applied twice;
// Givens rotations on the Hessenberg matrix; relative residual estimate
// |g_{j+1}| / ||b||; the preconditioned vectors Z are kept and x = Z y
// (flexible GMRES; for the fixed inner preconditioner this equals right-
// preconditioned GMRES).  An estimate <= 1e-15 ends the loop in every mode.
#include "ls_internal.h"

#include <chrono>
#include <cmath>
#include <complex>
#include <cstring>
#include <new>
#include <thread>
#include <type_traits>

namespace {
thread_local std::string g_last_error;

using zc = std::complex<double>;

inline zc toz(cplx a) { return zc(a.x, a.y); }
inline cplx fromz(zc a) { return cmk(a.real(), a.imag()); }

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) == hipSuccess && prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

// Grows a Krylov set to hold nvec vectors of `stride` elements each,
// keeping its contents (capacity doubles; the old block is released).
template <typename T>
ls_status ensure_krylov(ls_plan* p, KrylovSpaceT<T>& K, int nvec, size_t stride) {
  if (K.cap >= nvec) return LS_OK;
  const int ncap = std::max(nvec, std::max(4, 2 * K.cap));
  T* nb = nullptr;
  LS_TRY(plan_alloc(p, (void**)&nb, sizeof(T) * stride * ncap));
  if (K.base) {
    LS_HIP(hipMemcpyAsync(nb, K.base, sizeof(T) * stride * K.cap, hipMemcpyDeviceToDevice, p->stream));
    LS_HIP(hipStreamSynchronize(p->stream));
    for (auto it = p->allocs.begin(); it != p->allocs.end(); ++it)
      if (*it == K.base) {
        p->allocs.erase(it);
        break;
      }
    LS_HIP(hipFree(K.base));
  }
  K.base = nb;
  K.cap = ncap;
  return LS_OK;
}

struct GmresResult {
  int iters = 0;
  double relres = 0.0;
  bool converged = false;
};

// Flexible GMRES on B right-hand sides in lockstep (each with its own Krylov
// space, Hessenberg matrix and stopping test; vectors [B][N] of type T, the
// Krylov index slowest).  op and prec are callables (in, out, B) -> status.
// Inner products and the Hessenberg least squares are FP64.  A right-hand
// side that has converged keeps a zero next basis vector, so it costs work
// but never divides by zero.
template <typename T, class Op, class Prec>
ls_status fgmres(ls_plan* p, Op op, Prec prec, const T* b, T* x, int B, double tol, int maxit,
                 int fixed, KrylovSpaceT<T>& KV, KrylovSpaceT<T>& KZ, std::vector<GmresResult>& res) {
  const size_t N = (size_t)p->n * p->n;
  // Krylov index stride: always max_batch vectors, so a set allocated for one
  // call fits every later call whatever its B
  const size_t stride = (size_t)p->opt.max_batch * N;
  const int limit = fixed > 0 ? fixed : maxit;
  res.assign(B, GmresResult{});
  std::vector<double> beta(B), hn(B), sc(B);
  LS_TRY(vec_norms(p, b, N, B, beta.data()));
  std::vector<char> active(B);
  int nactive = 0;
  for (int i = 0; i < B; ++i) {
    active[i] = beta[i] > 0.0;
    nactive += active[i];
    if (!active[i]) {  // zero right-hand side: x = 0 is exact; NaN: not converged
      res[i].converged = beta[i] == 0.0;
      res[i].relres = beta[i] == 0.0 ? 0.0 : beta[i];
    }
    sc[i] = active[i] ? 1.0 / beta[i] : 0.0;
  }
  if (nactive == 0) return vec_zero(p, x, (size_t)B * N);
  LS_TRY(ensure_krylov(p, KV, 2, stride));
  LS_TRY(ensure_krylov(p, KZ, 1, stride));
  LS_TRY(vec_scale_b(p, KV.base, b, sc.data(), N, B));
  std::vector<std::vector<std::vector<zc>>> H(B);  // [b][column]
  std::vector<std::vector<double>> cs(B);
  std::vector<std::vector<zc>> sn(B), gv(B);
  for (int i = 0; i < B; ++i) gv[i].assign(1, zc(beta[i], 0.0));
  std::vector<cplx> h1, h2;
  int jlast = 0;
  for (int j = 0; j < limit; ++j) {
    LS_TRY(ensure_krylov(p, KV, j + 2, stride));
    LS_TRY(ensure_krylov(p, KZ, j + 1, stride));
    T* Vj = KV.base + (size_t)j * stride;
    T* Zj = KZ.base + (size_t)j * stride;
    T* w = KV.base + (size_t)(j + 1) * stride;
    LS_TRY(prec(Vj, Zj, B));
    LS_TRY(op(Zj, w, B));
    h1.resize((size_t)B * (j + 1));
    h2.resize((size_t)B * (j + 1));
    if (j + 1 <= 8) {  // fused on the device, one transfer
      LS_TRY(vec_cgs2(p, KV.base, j + 1, stride, w, N, B, h1.data(), h2.data(), hn.data()));
      for (int i = 0; i < B; ++i)  // NaN stays NaN: a poisoned vector must not look converged
        hn[i] = std::isnan(hn[i]) ? hn[i] : std::sqrt(std::fmax(hn[i], 0.0));
    } else {
      LS_TRY(vec_multidot(p, KV.base, j + 1, stride, w, N, B, h1.data()));
      LS_TRY(vec_multiaxpy(p, w, KV.base, j + 1, stride, h1.data(), N, B));
      LS_TRY(vec_multidot(p, KV.base, j + 1, stride, w, N, B, h2.data()));
      LS_TRY(vec_multiaxpy(p, w, KV.base, j + 1, stride, h2.data(), N, B));
      LS_TRY(vec_norms(p, w, N, B, hn.data()));
    }
    jlast = j + 1;
    for (int i = 0; i < B; ++i) {
      if (!active[i]) continue;
      std::vector<zc> col(j + 2);
      for (int k = 0; k <= j; ++k)
        col[k] = toz(h1[(size_t)i * (j + 1) + k]) + toz(h2[(size_t)i * (j + 1) + k]);
      col[j + 1] = zc(hn[i], 0.0);
      for (int k = 0; k < j; ++k) {
        const zc a0 = col[k], b0 = col[k + 1];
        col[k] = cs[i][k] * a0 + sn[i][k] * b0;
        col[k + 1] = -std::conj(sn[i][k]) * a0 + cs[i][k] * b0;
      }
      const zc a0 = col[j];
      const double bb = col[j + 1].real();
      const double r = std::hypot(std::abs(a0), bb);
      double c;
      zc s;
      if (std::abs(a0) == 0.0) {
        c = 0.0;
        s = zc(1.0, 0.0);
        col[j] = zc(bb, 0.0);
      } else {
        const zc ph = a0 / std::abs(a0);
        c = std::abs(a0) / r;
        s = ph * bb / r;
        col[j] = ph * r;
      }
      col[j + 1] = 0.0;
      cs[i].push_back(c);
      sn[i].push_back(s);
      gv[i].push_back(-std::conj(s) * gv[i][j]);
      gv[i][j] = c * gv[i][j];
      H[i].push_back(col);
      const double rel = std::abs(gv[i][j + 1]) / beta[i];
      res[i].iters = j + 1;
      res[i].relres = rel;
      res[i].converged = rel <= tol;
      // stop: converged, Krylov space exhausted, or a non-finite value
      // (the right-hand side stays unconverged)
      if ((fixed == 0 && rel <= tol) || rel <= 1e-15 || hn[i] == 0.0 || !std::isfinite(rel)) {
        active[i] = 0;
        --nactive;
      }
    }
    if (nactive == 0 || j + 1 == limit) break;
    for (int i = 0; i < B; ++i) sc[i] = (active[i] && hn[i] > 0.0) ? 1.0 / hn[i] : 0.0;
    LS_TRY(vec_scale_b(p, w, w, sc.data(), N, B));
  }
  // R y = g per right-hand side, padded with zeros to jlast columns
  std::vector<cplx> yc((size_t)B * jlast, cmk(0.0, 0.0));
  for (int i = 0; i < B; ++i) {
    const int jd = (int)H[i].size();
    std::vector<zc> y(jd);
    for (int r = jd - 1; r >= 0; --r) {
      zc s = gv[i][r];
      for (int k = r + 1; k < jd; ++k) s -= H[i][k][r] * y[k];
      y[r] = s / H[i][r][r];
    }
    for (int k = 0; k < jd; ++k) yc[(size_t)i * jlast + k] = fromz(y[k]);
  }
  return vec_lincomb(p, x, KZ.base, jlast, stride, yc.data(), N, B);
}

template <typename T>
ls_status inner_prec_eager(ls_plan* p, const T* in, T* out, int B) {
  const size_t N = (size_t)p->n * p->n;
  switch (p->opt.precond) {
    case LS_PREC_BD:
      return bidirectional_apply(p, in, out, B);
    case LS_PREC_PT1:
      return sweep_apply(p, 0, in, out, false, B);
    default:
      return vec_copy(p, out, in, N * B);
  }
}

// The inner preconditioner (Alg. 2 or Alg. 1) is a fixed sequence of
// kernels and device copies for given (in, out, B): it is captured once into
// a hipGraph and replayed.  Nothing in it synchronises or sets memory with
// memset nodes; the graph only references plan-owned buffers besides in/out.
template <typename T>
ls_status inner_prec(ls_plan* p, const T* in, T* out, int B) {
  if (!p->opt.use_graphs || p->opt.precond == LS_PREC_NONE)
    return inner_prec_eager<T>(p, in, out, B);
  for (auto& g : p->graphs)
    if (g.in == (const void*)in && g.out == (void*)out && g.B == B && g.elem == (int)sizeof(T)) {
      LS_HIP(hipGraphLaunch(g.exec, p->stream));
      return LS_OK;
    }
  LS_HIP(hipStreamBeginCapture(p->stream, hipStreamCaptureModeRelaxed));
  ls_status st = inner_prec_eager<T>(p, in, out, B);
  hipGraph_t graph = nullptr;
  hipError_t e = hipStreamEndCapture(p->stream, &graph);
  if (st != LS_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return st;
  }
  if (e != hipSuccess) {
    ls_set_error(std::string("graph capture failed: ") + hipGetErrorString(e));
    return LS_EDEVICE;
  }
  hipGraphExec_t exec = nullptr;
  e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) {
    ls_set_error(std::string("graph instantiate failed: ") + hipGetErrorString(e));
    return LS_EDEVICE;
  }
  if (p->graphs.size() >= 64) {
    (void)hipGraphExecDestroy(p->graphs.front().exec);
    p->graphs.erase(p->graphs.begin());
  }
  p->graphs.push_back(GraphEntry{(const void*)in, (void*)out, B, (int)sizeof(T), exec});
  LS_HIP(hipGraphLaunch(exec, p->stream));
  return LS_OK;
}

template <typename T>
struct PK;
template <>
struct PK<cplx> {
  static cplx*& rhs(ls_plan* p) { return p->inner_rhs; }
  static KrylovSpaceT<cplx>& iV(ls_plan* p) { return p->innerV; }
  static KrylovSpaceT<cplx>& iZ(ls_plan* p) { return p->innerZ; }
  static KrylovSpaceT<cplx>& oV(ls_plan* p) { return p->outerV; }
  static KrylovSpaceT<cplx>& oZ(ls_plan* p) { return p->outerZ; }
};
template <>
struct PK<fcplx> {
  static fcplx*& rhs(ls_plan* p) { return p->inner_rhs32; }
  static KrylovSpaceT<fcplx>& iV(ls_plan* p) { return p->innerV32; }
  static KrylovSpaceT<fcplx>& iZ(ls_plan* p) { return p->innerZ32; }
  static KrylovSpaceT<fcplx>& oV(ls_plan* p) { return p->outerV32; }
  static KrylovSpaceT<fcplx>& oZ(ls_plan* p) { return p->outerZ32; }
};

// Alg. 3 for B right-hand sides, in the precision of T.
template <typename T>
ls_status precond_batch(ls_plan* p, const T* r, T* z, int B, std::vector<GmresResult>& res) {
  const size_t N = (size_t)p->n * p->n;
  T*& g = PK<T>::rhs(p);
  if (!g) LS_TRY(plan_alloc(p, (void**)&g, sizeof(T) * N * p->opt.max_batch));
  LS_TRY(stencil_apply_A(p, r, g, B));
  if (p->opt.inner_fixed_iters == 1) {
    // one inner iteration (Section 6: the inner solve relaxed under the
    // flexible outer loop) in closed form, with no host transfer: zt = M g,
    // w = C zt, z = ((w^H g) / (w^H w)) zt -- the value one step of the
    // right-preconditioned GMRES below gives, up to rounding (M is linear)
    KrylovSpaceT<T>& KV = PK<T>::iV(p);
    KrylovSpaceT<T>& KZ = PK<T>::iZ(p);
    const size_t stride = (size_t)p->opt.max_batch * N;
    LS_TRY(ensure_krylov(p, KV, 1, stride));
    LS_TRY(ensure_krylov(p, KZ, 1, stride));
    LS_TRY(inner_prec<T>(p, g, KZ.base, B));
    LS_TRY(stencil_apply_C(p, KZ.base, KV.base, B));
    LS_TRY(vec_minres_scale(p, KV.base, g, KZ.base, z, N, B));
    GmresResult one;
    one.iters = 1;
    res.assign(B, one);
    return LS_OK;
  }
  auto op = [&](const T* in, T* out, int nb) { return stencil_apply_C(p, in, out, nb); };
  auto pr = [&](const T* in, T* out, int nb) { return inner_prec<T>(p, in, out, nb); };
  return fgmres<T>(p, op, pr, g, z, B, p->opt.inner_tol, p->opt.max_inner,
                   p->opt.inner_fixed_iters, PK<T>::iV(p), PK<T>::iZ(p), res);
}

__global__ void k_real_to_f32(const double* __restrict__ a, float* __restrict__ b, size_t cnt) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < cnt) b[i] = (float)a[i];
}

// Runs fn on FP32 copies of FP64 device arrays (FP32 plans).
struct F32Scratch {
  fcplx* a = nullptr;
  fcplx* b = nullptr;
};

ls_status f32_scratch(ls_plan* p, F32Scratch& s) {
  // vtmp32 holds 3 batches of grid vectors; slots 1 and 2 are free outside
  // Alg. 2's residual (slot 0)
  const size_t BN = (size_t)p->n * p->n * p->opt.max_batch;
  s.a = p->vtmp32 + BN;
  s.b = p->vtmp32 + 2 * BN;
  return LS_OK;
}

bool valid_opts(const ls_options& o) {
  if (o.use_graphs < 0 || o.use_graphs > 1 || o.autotune < 0 || o.autotune > 1) return false;
  if (o.fft_variant < 0 || o.fft_variant >= kFftVariants) return false;
  if (o.sweep != LS_SWEEP_SEQUENTIAL && o.sweep != LS_SWEEP_DECOUPLED) return false;
  if (o.level0 != LS_LEVEL0_AUTO && o.level0 != LS_LEVEL0_DENSE) return false;
  return o.ext >= 0 && o.inner_tol > 0 && o.max_outer >= 1 && o.max_inner >= 1 &&
         (o.precision == LS_FP64 || o.precision == LS_FP32_REFINE) && o.precond >= LS_PREC_BD &&
         o.precond <= LS_PREC_NONE && o.inner_fixed_iters >= 0 && o.max_batch >= 1 &&
         o.slabs >= 0 && std::isfinite(o.shift_c) && o.lowp_tol > 0 && o.max_refine >= 1;
}

}  // namespace

void ls_set_error(const std::string& msg) { g_last_error = msg; }

double plan_clock_ms(ls_plan* p) {
  (void)hipStreamSynchronize(p->stream);
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

ls_status plan_alloc(ls_plan* p, void** ptr, size_t bytes) {
  *ptr = nullptr;
  if (bytes == 0) bytes = 16;
  hipError_t e = hipMalloc(ptr, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    ls_set_error("hipMalloc of " + std::to_string(bytes) + " bytes failed: " + hipGetErrorString(e));
    *ptr = nullptr;
    return LS_ENOMEM;
  }
  p->allocs.push_back(*ptr);
  return LS_OK;
}

// Runs an FP32 operation on B grid vectors given and returned in FP64
// (FP32 plans).
template <class F>
static ls_status via_f32(ls_plan* p, const double* in, double* out, int B, F fn) {
  const size_t N = (size_t)p->n * p->n;
  F32Scratch sc;
  LS_TRY(f32_scratch(p, sc));
  std::vector<double> one(B, 1.0);
  LS_TRY(vec_to_f32_b(p, sc.a, reinterpret_cast<const cplx*>(in), one.data(), N, B));
  LS_TRY(fn(sc.a, sc.b));
  return vec_from_f32_b(p, reinterpret_cast<cplx*>(out), nullptr, sc.b, one.data(), N, B);
}

// Outer flexible GMRES in the precision of T on H u = f for B right-hand sides.
template <typename T>
static ls_status outer_fgmres(ls_plan* p, const T* f, T* u, int B, const std::vector<double>& tol,
                              std::vector<GmresResult>& res, std::vector<int>& inner_total) {
  auto op = [&](const T* in, T* out, int nb) -> ls_status {
    if constexpr (std::is_same<T, cplx>::value) return apply_H(p, in, out, nb, 1.0, 1.0);
    else return apply_H32(p, in, out, nb, 1.0, 1.0);
  };
  auto pr = [&](const T* in, T* out, int nb) -> ls_status {
    std::vector<GmresResult> r;
    ls_status s = precond_batch<T>(p, in, out, nb, r);
    for (int i = 0; i < nb; ++i) inner_total[i] += r[i].iters;
    return s;
  };
  // one tolerance for the lockstep loop: the largest requested (the others
  // are met when the loop continues for the slowest right-hand side)
  double t = 0.0;
  for (double x : tol) t = std::max(t, x);
  return fgmres<T>(p, op, pr, f, u, B, t, p->opt.max_outer, 0, PK<T>::oV(p), PK<T>::oZ(p), res);
}

// r = f - H u and ||r|| / ||f|| per right-hand side, FP64.
static ls_status true_residual(ls_plan* p, const cplx* f, const cplx* u, cplx* r, int B,
                               const std::vector<double>& nf, std::vector<double>& rel) {
  const size_t N = (size_t)p->n * p->n;
  std::vector<double> nr(B);
  LS_TRY(apply_H(p, u, r, B, 1.0, 1.0));
  LS_TRY(vec_axpy(p, r, f, cmk(-1.0, 0.0), N * B));   // r = H u - f
  LS_TRY(vec_scale_copy(p, r, r, -1.0, N * B));       // r = f - H u
  LS_TRY(vec_norms(p, r, N, B, nr.data()));
  rel.resize(B);
  for (int i = 0; i < B; ++i) rel[i] = nf[i] > 0 ? nr[i] / nf[i] : 0.0;
  return LS_OK;
}


// ------------------------------------------------------- correction solves
// X = u + back_i d_i with d_i ~ H^{-1} (scale_i r_i): flexible GMRES in the
// plan's precision (at most maxit iterations, relative tolerance tgt) with
// the preconditioner pr64 (FP64 plans) or pr32 (FP32 plans).  A right-hand
// side with scale 0 gets d = 0.  X must not alias u or r.
template <class Pr64, class Pr32>
static ls_status correction(ls_plan* p, const cplx* r, const cplx* u, cplx* X, int B,
                            const std::vector<double>& scale, const std::vector<double>& back,
                            double tgt, int maxit, Pr64 pr64, Pr32 pr32,
                            std::vector<GmresResult>& res) {
  const size_t N = (size_t)p->n * p->n;
  if (p->fp32) {
    F32Scratch sc;
    LS_TRY(f32_scratch(p, sc));
    LS_TRY(vec_to_f32_b(p, sc.a, r, scale.data(), N, B));
    auto op = [&](const fcplx* in, fcplx* out, int nb) { return apply_H32(p, in, out, nb, 1.0, 1.0); };
    LS_TRY(fgmres<fcplx>(p, op, pr32, sc.a, sc.b, B, tgt, maxit, 0, p->outerV32, p->outerZ32, res));
    return vec_from_f32_b(p, X, u, sc.b, back.data(), N, B);
  }
  // vtmp slot 2 is free outside ls_solve's own loop (slot 0 is Alg. 2's
  // residual, slot 1 the solve's residual)
  cplx* rs = p->vtmp + 2 * (size_t)p->opt.max_batch * N;
  LS_TRY(vec_scale_b(p, rs, r, scale.data(), N, B));
  auto op = [&](const cplx* in, cplx* out, int nb) { return apply_H(p, in, out, nb, 1.0, 1.0); };
  LS_TRY(fgmres<cplx>(p, op, pr64, rs, X, B, tgt, maxit, 0, p->outerV, p->outerZ, res));
  LS_TRY(vec_scale_b(p, X, X, back.data(), N, B));
  return vec_axpy(p, X, u, cmk(1.0, 0.0), N * B);
}

// Scales of one refinement step: active right-hand sides (rel > tol) get
// their residual normalised and a target max(floor, 0.5 tol / rel); the
// lockstep loop runs to the smallest target.
static double refine_scales(const std::vector<double>& rel, const std::vector<double>& nf, double tol,
                            double floor, std::vector<double>& scale, std::vector<double>& back) {
  const int B = (int)rel.size();
  scale.assign(B, 0.0);
  back.assign(B, 0.0);
  double tmin = 1.0;
  for (int i = 0; i < B; ++i) {
    if (!(rel[i] > tol)) continue;
    const double nr = rel[i] * nf[i];
    scale[i] = 1.0 / nr;
    back[i] = nr;
    tmin = std::min(tmin, std::max(floor, 0.5 * tol / rel[i]));
  }
  return tmin;
}

// Iterative refinement with the plan's two-level preconditioner from the
// state (u, r = f - H u, rel = ||r|| / ||f||) until rel <= tol for every
// right-hand side or max_refine steps; X is scratch for the candidate u.
static ls_status refine_bd(ls_plan* p, const cplx* fb, cplx* ub, cplx* rbuf, cplx* X, int B, double tol,
                           const std::vector<double>& nf, std::vector<double>& rel,
                           std::vector<int>& outer_total, std::vector<int>& inner_total) {
  const size_t N = (size_t)p->n * p->n;
  auto bd = [&](auto tag) {
    using T = decltype(tag);
    return [&, p](const T* in, T* out, int nb) -> ls_status {
      std::vector<GmresResult> r;
      ls_status st = precond_batch<T>(p, in, out, nb, r);
      for (int i = 0; i < nb; ++i) inner_total[i] += r[i].iters;
      return st;
    };
  };
  for (int it = 0; it < p->opt.max_refine; ++it) {
    std::vector<double> scale, back;
    const double tgt = refine_scales(rel, nf, tol, p->fp32 ? p->opt.lowp_tol : 0.0, scale, back);
    bool done = true;
    for (int i = 0; i < B; ++i) done = done && !(rel[i] > tol);
    if (done) break;
    std::vector<GmresResult> res;
    LS_TRY(correction(p, rbuf, ub, X, B, scale, back, tgt, p->opt.max_outer, bd(cplx{}), bd(fcplx{}), res));
    for (int i = 0; i < B; ++i) outer_total[i] += scale[i] > 0 ? res[i].iters : 0;
    LS_TRY(vec_copy(p, ub, X, N * B));
    LS_TRY(true_residual(p, fb, ub, rbuf, B, nf, rel));
  }
  return LS_OK;
}

// Sets the stream of a network handle for the lifetime of a solve.
struct FnoStreamGuard {
  ls_fno* f;
  hipStream_t old;
  FnoStreamGuard(ls_fno* f_, hipStream_t s) : f(f_), old(fno_swap_stream(f_, s)) {}
  ~FnoStreamGuard() { fno_swap_stream(f, old); }
};

extern "C" {

void ls_options_default(ls_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->slabs = 0;
  o->ext = 10;
  o->inner_tol = 1e-3;
  o->max_outer = 100;
  o->max_inner = 50;
  o->shift_c = 0.0;
  o->precision = LS_FP64;
  o->precond = LS_PREC_BD;
  o->inner_fixed_iters = 0;
  o->max_batch = 1;
  o->lowp_tol = 1e-5;
  o->max_refine = 10;
  o->use_graphs = 1;
  o->autotune = 1;
  o->fft_variant = 0;
  o->sweep = LS_SWEEP_SEQUENTIAL;
  o->level0 = LS_LEVEL0_AUTO;
}

const char* ls_status_str(ls_status s) {
  switch (s) {
    case LS_OK: return "LS_OK";
    case LS_EINVAL: return "LS_EINVAL";
    case LS_ENOMEM: return "LS_ENOMEM";
    case LS_EDEVICE: return "LS_EDEVICE";
    case LS_ENOCONV: return "LS_ENOCONV";
    case LS_ESINGULAR: return "LS_ESINGULAR";
    case LS_EUNSUPPORTED: return "LS_EUNSUPPORTED";
  }
  return "LS_UNKNOWN";
}

const char* ls_last_error(void) { return g_last_error.c_str(); }

ls_status ls_plan_destroy(ls_plan* p) {
  if (!p) return LS_OK;
  DeviceGuard dg(p->device);
  (void)hipStreamSynchronize(p->stream);
  for (auto& g : p->graphs) (void)hipGraphExecDestroy(g.exec);
  for (void* a : p->allocs) (void)hipFree(a);
  if (p->hres) (void)hipHostFree(p->hres);
  if (p->hcoef) (void)hipHostFree(p->hcoef);
  if (p->coef_ev) (void)hipEventDestroy(p->coef_ev);
  for (int k = 0; k < ls_plan::kSide; ++k) {
    if (p->side[k]) (void)hipStreamDestroy(p->side[k]);
    if (p->side_join[k]) (void)hipEventDestroy(p->side_join[k]);
  }
  if (p->side_fork) (void)hipEventDestroy(p->side_fork);
  if (p->own_stream) (void)hipStreamDestroy(p->stream);
  delete p;
  return LS_OK;
}

// The off-line stage (Section 4.1).  With src, a plan of the same (n, h,
// omega) -- whose kernel samples, spectrum and stencils do not depend on the
// medium -- the spectrum and stencil tables are copied from it instead of
// recomputed, and its autotuned FFT variants are reused.
static ls_status create_impl(ls_plan* p, const double* m, const ls_plan* src) {
  const int n = p->n;
  const double t_start = plan_clock_ms(p);
  LS_TRY(plan_alloc(p, (void**)&p->m, sizeof(double) * n * n));
  LS_HIP(hipMemcpyAsync(p->m, m, sizeof(double) * n * n, hipMemcpyDeviceToDevice, p->stream));
  LS_TRY(fft_setup_twiddles(p));
  LS_TRY(plan_alloc(p, (void**)&p->stencil_d, sizeof(cplx) * 324));
  LS_TRY(plan_alloc(p, (void**)&p->spec, sizeof(cplx) * p->spec_side * p->spec_side));
  if (p->fp32) {
    LS_TRY(plan_alloc(p, (void**)&p->f32.m, sizeof(float) * n * n));
    k_real_to_f32<<<(unsigned)(((size_t)n * n + 255) / 256), 256, 0, p->stream>>>(p->m, p->f32.m,
                                                                                (size_t)n * n);
    LS_HIP(hipGetLastError());
    LS_TRY(plan_alloc(p, (void**)&p->f32.stencil, sizeof(fcplx) * 324));
    LS_TRY(plan_alloc(p, (void**)&p->f32.spec, sizeof(fcplx) * p->spec_side * p->spec_side));
    LS_TRY(plan_alloc(p, (void**)&p->f32.fft_work, sizeof(fcplx) * (size_t)p->opt.max_batch * n * p->P));
    LS_TRY(plan_alloc(p, (void**)&p->vtmp32, sizeof(fcplx) * (size_t)3 * n * n * p->opt.max_batch));
  }
  if (src) {
    const size_t ss = (size_t)p->spec_side * p->spec_side;
    LS_HIP(hipMemcpyAsync(p->spec, src->spec, sizeof(cplx) * ss, hipMemcpyDeviceToDevice, p->stream));
    LS_HIP(hipMemcpyAsync(p->stencil_d, src->stencil_d, sizeof(cplx) * 324, hipMemcpyDeviceToDevice, p->stream));
    std::memcpy(p->alpha_h, src->alpha_h, sizeof(p->alpha_h));
    std::memcpy(p->beta_h, src->beta_h, sizeof(p->beta_h));
    if (p->fp32) {
      LS_TRY(stencils_to_f32(p));
      LS_TRY(spectrum_to_f32(p));
    }
    p->stage_ms[2] = plan_clock_ms(p) - t_start;
  } else {
    cplx* circ = nullptr;
    LS_HIP(hipMalloc(&circ, sizeof(cplx) * (size_t)p->P * p->P));
    double t0 = plan_clock_ms(p), t1 = t0, t2 = t0;
    ls_status s = launch_circulant(p, circ);
    if (s == LS_OK) {
      t1 = plan_clock_ms(p);
      s = stencils_build(p, circ);
    }
    if (s == LS_OK && p->fp32) s = stencils_to_f32(p);
    if (s == LS_OK) {
      t2 = plan_clock_ms(p);
      s = fft2_full_forward(p, circ);
    }
    if (s == LS_OK) s = spectrum_extract(p, circ);
    if (s == LS_OK && hipStreamSynchronize(p->stream) != hipSuccess) s = LS_EDEVICE;
    (void)hipFree(circ);
    if (s != LS_OK) return s;
    const double t3 = plan_clock_ms(p);
    p->stage_ms[0] = t1 - t0;
    p->stage_ms[1] = t2 - t1;
    p->stage_ms[2] = t3 - t2;
  }
  LS_TRY(plan_alloc(p, (void**)&p->fft_work, sizeof(cplx) * (size_t)p->opt.max_batch * n * p->P));
  LS_TRY(plan_alloc(p, (void**)&p->vtmp, sizeof(cplx) * (size_t)3 * n * n * p->opt.max_batch));
  if (p->opt.precond != LS_PREC_NONE) LS_TRY(slabs_build(p));
  p->col_variant64 = p->col_variant32 = p->opt.fft_variant;
  const double t_tune = plan_clock_ms(p);
  bool tuned = false;
  if (p->opt.autotune) {
    if (src && src->opt.autotune && src->fp32 == p->fp32) {
      p->col_variant64 = src->col_variant64;
      p->col_variant32 = src->col_variant32;
      std::memcpy(p->tune_ms64, src->tune_ms64, sizeof(p->tune_ms64));
      std::memcpy(p->tune_ms32, src->tune_ms32, sizeof(p->tune_ms32));
    } else {
      LS_TRY(fft_autotune(p));
      tuned = true;
    }
  }
  LS_HIP(hipStreamSynchronize(p->stream));
  const double t_end = plan_clock_ms(p);
  p->stage_ms[7] = tuned ? t_end - t_tune : 0.0;
  p->stage_ms[8] = t_end - t_start;
  return LS_OK;
}

// Validates the arguments and sets up a plan's geometry, device and stream;
// the off-line stage itself is create_impl.
static ls_status create_common(ls_plan** out, int n, double h, double omega, const double* m,
                               const ls_options* opt, void* stream, const ls_plan* src) {
  if (!out || !m) {
    ls_set_error("ls_plan_create: null pointer");
    return LS_EINVAL;
  }
  *out = nullptr;
  ls_options o;
  ls_options_default(&o);
  if (opt) o = *opt;
  if (n < 8 || 2 * n - 1 > 4096 || !(h > 0) || !(omega > 0) || !std::isfinite(h) ||
      !std::isfinite(omega) || !valid_opts(o)) {
    ls_set_error("ls_plan_create: invalid size, h, omega or options");
    return LS_EINVAL;
  }
  int L = o.slabs > 0 ? o.slabs : std::max(1, n / 64);
  if (L > n / 2 && L > 1) {
    ls_set_error("ls_plan_create: too many slabs for n");
    return LS_EINVAL;
  }
  if (L > 1 && (o.ext < 1 || n / L < 1)) {
    ls_set_error("ls_plan_create: layers need ext >= 1");
    return LS_EINVAL;
  }
  ls_plan* p = new (std::nothrow) ls_plan();
  if (!p) return LS_ENOMEM;
  p->n = n;
  p->h = h;
  p->omega = omega;
  p->opt = o;
  p->L = L;
  p->fp32 = (o.precision == LS_FP32_REFINE);
  p->stream = reinterpret_cast<hipStream_t>(stream);
  int P = 1, logP = 0;
  while (P < 2 * n - 1) { P <<= 1; ++logP; }
  p->P = P;
  p->logP = logP;
  p->spec_side = P / 2 + 1;
  if (hipGetDevice(&p->device) != hipSuccess) {
    ls_set_error("ls_plan_create: no HIP device");
    delete p;
    return LS_EDEVICE;
  }
  // the allocation-free entry point's static scratch: its device address on
  // this device, taken once with the device current
  if (ls_status ss = static_scratch_init(p->device); ss != LS_OK) {
    delete p;
    return ss;
  }
  if (hipDeviceGetAttribute(&p->cus, hipDeviceAttributeMultiprocessorCount, p->device) != hipSuccess ||
      p->cus < 1)
    p->cus = 256;
  if (p->stream == nullptr) {
    // a private blocking stream: ordered with the null stream like it, but
    // capturable into graphs
    if (hipStreamCreate(&p->stream) != hipSuccess) {
      ls_set_error("ls_plan_create: stream creation failed");
      delete p;
      return LS_EDEVICE;
    }
    p->own_stream = true;
  }
  ls_status s = create_impl(p, m, src);
  if (s != LS_OK) {
    std::string keep = g_last_error;
    ls_plan_destroy(p);
    g_last_error = keep;
    return s;
  }
  *out = p;
  return LS_OK;
}

ls_status ls_plan_create(ls_plan** out, int n, double h, double omega, const double* m,
                         const ls_options* opt, void* stream) {
  return create_common(out, n, h, omega, m, opt, stream, nullptr);
}

ls_status ls_plan_create_like(ls_plan** out, const ls_plan* src, const double* m, const ls_options* opt,
                              void* stream) {
  if (!src) {
    ls_set_error("ls_plan_create_like: null source plan");
    return LS_EINVAL;
  }
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != src->device) {
    ls_set_error("ls_plan_create_like: the source plan lives on another device");
    return LS_EINVAL;
  }
  return create_common(out, src->n, src->h, src->omega, m, opt, stream, src);
}

ls_status ls_plan_timings(const ls_plan* p, double* ms, int count) {
  if (!p || !ms || count < 1) {
    ls_set_error("ls_plan_timings: bad arguments");
    return LS_EINVAL;
  }
  for (int i = 0; i < count && i < 9; ++i) ms[i] = p->stage_ms[i];
  for (int i = 9; i < count; ++i) ms[i] = 0.0;
  return LS_OK;
}

ls_status ls_plan_info(const ls_plan* p, int* info, int count) {
  if (!p || !info || count < 1) {
    ls_set_error("ls_plan_info: bad arguments");
    return LS_EINVAL;
  }
  int top_blocks = 0;  // blocks of the first slab's dense top operator (0: none)
  if (!p->slabs[0].empty() && p->slabs[0][0].top_level >= 1)
    top_blocks = p->slabs[0][0].levels[p->slabs[0][0].top_level].nl;
  const int v[4] = {p->tri_ok ? 1 : 0, top_blocks, p->col_variant64, p->fp32 ? p->col_variant32 : -1};
  for (int i = 0; i < count; ++i) info[i] = i < 4 ? v[i] : 0;
  return LS_OK;
}

ls_status ls_plan_dims(const ls_plan* p, int* P, int* L, int* spec_side) {
  if (!p) return LS_EINVAL;
  if (P) *P = p->P;
  if (L) *L = p->L;
  if (spec_side) *spec_side = p->spec_side;
  return LS_OK;
}

ls_status ls_apply(ls_plan* p, const double* v, double* Hv, int batch) {
  if (!p || !v || !Hv || batch < 1 || batch > p->opt.max_batch) {
    ls_set_error("ls_apply: bad arguments (batch must be in [1, max_batch])");
    return LS_EINVAL;
  }
  DeviceGuard dg(p->device);
  return apply_H(p, reinterpret_cast<const cplx*>(v), reinterpret_cast<cplx*>(Hv), batch, 1.0, 1.0);
}

ls_status ls_rhs_from_incident(ls_plan* p, const double* uI, double* f, int batch) {
  if (!p || !uI || !f || batch < 1 || batch > p->opt.max_batch) {
    ls_set_error("ls_rhs_from_incident: bad arguments");
    return LS_EINVAL;
  }
  DeviceGuard dg(p->device);
  return apply_H(p, reinterpret_cast<const cplx*>(uI), reinterpret_cast<cplx*>(f), batch, 0.0, -1.0);
}

ls_status ls_get_kernel_samples(ls_plan* p, double* w) {
  if (!p || !w) return LS_EINVAL;
  DeviceGuard dg(p->device);
  return launch_kernel_samples(p, reinterpret_cast<cplx*>(w));
}

ls_status ls_get_spectrum(ls_plan* p, double* S) {
  if (!p || !S) return LS_EINVAL;
  DeviceGuard dg(p->device);
  LS_HIP(hipMemcpyAsync(S, p->spec, sizeof(cplx) * p->spec_side * p->spec_side,
                        hipMemcpyDeviceToDevice, p->stream));
  return LS_OK;
}

ls_status ls_get_stencils(ls_plan* p, double* alpha, double* beta) {
  if (!p || !alpha || !beta) return LS_EINVAL;
  std::memcpy(alpha, p->alpha_h, sizeof(p->alpha_h));
  std::memcpy(beta, p->beta_h, sizeof(p->beta_h));
  return LS_OK;
}

ls_status ls_stencil_A(ls_plan* p, const double* r, double* y, int batch) {
  if (!p || !r || !y || batch < 1 || r == y) return LS_EINVAL;
  DeviceGuard dg(p->device);
  return stencil_apply_A(p, reinterpret_cast<const cplx*>(r), reinterpret_cast<cplx*>(y), batch);
}

ls_status ls_stencil_C(ls_plan* p, const double* v, double* y, int batch) {
  if (!p || !v || !y || batch < 1 || v == y) return LS_EINVAL;
  DeviceGuard dg(p->device);
  return stencil_apply_C(p, reinterpret_cast<const cplx*>(v), reinterpret_cast<cplx*>(y), batch);
}

ls_status ls_slab_info(const ls_plan* p, int orient, int slab, int* lims) {
  if (!p || !lims || orient < 0 || orient > 1 || slab < 0 || slab >= p->L ||
      p->slabs[orient].empty()) {
    ls_set_error("ls_slab_info: bad arguments");
    return LS_EINVAL;
  }
  const Slab& s = p->slabs[orient][slab];
  lims[0] = s.a;
  lims[1] = s.b;
  lims[2] = s.z0;
  lims[3] = s.z1;
  return LS_OK;
}

ls_status ls_slab_solve(ls_plan* p, int orient, int slab, const double* b, double* x) {
  if (!p || !b || !x || orient < 0 || orient > 1 || slab < 0 || slab >= p->L ||
      p->slabs[orient].empty()) {
    ls_set_error("ls_slab_solve: bad arguments");
    return LS_EINVAL;
  }
  DeviceGuard dg(p->device);
  Slab& s = p->slabs[orient][slab];
  const size_t cnt = (size_t)p->n * s.q;
  const cplx* bb = reinterpret_cast<const cplx*>(b);
  cplx* xx = reinterpret_cast<cplx*>(x);
  const size_t BN = (size_t)p->n * p->n * p->opt.max_batch;  // n*q <= one slot
  if (p->fp32) {
    fcplx* gi = p->vtmp32;
    fcplx* yo = p->vtmp32 + BN;
    LS_TRY(vec_to_f32(p, gi, bb, 1.0, cnt));
    LS_TRY(slab_solve(p, s, gi, yo, 1));
    return vec_from_f32(p, xx, nullptr, yo, 1.0, cnt);
  }
  if (bb == xx) {  // in place: solve from a copy
    cplx* gi = p->vtmp;
    LS_TRY(vec_copy(p, gi, bb, cnt));
    return slab_solve(p, s, gi, xx, 1);
  }
  return slab_solve(p, s, bb, xx, 1);
}

ls_status ls_slab_solve_noalloc(ls_plan* p, int orient, int slab, const double* b, double* x) {
  if (!p || !b || !x || orient < 0 || orient > 1 || slab < 0 || slab >= p->L ||
      p->slabs[orient].empty()) {
    ls_set_error("ls_slab_solve_noalloc: bad arguments");
    return LS_EINVAL;
  }
  DeviceGuard dg(p->device);
  return slab_solve_noalloc(p, p->slabs[orient][slab], reinterpret_cast<const cplx*>(b),
                            reinterpret_cast<cplx*>(x));
}

size_t ls_noalloc_scratch_bytes(void) { return static_scratch_bytes(); }

ls_status ls_sweep(ls_plan* p, int orient, const double* g, double* v) {
  if (!p || !g || !v || g == v || orient < 0 || orient > 1 || p->slabs[orient].empty()) {
    ls_set_error("ls_sweep: bad arguments");
    return LS_EINVAL;
  }
  DeviceGuard dg(p->device);
  if (p->fp32)
    return via_f32(p, g, v, 1, [&](const fcplx* a, fcplx* b) { return sweep_apply(p, orient, a, b, false, 1); });
  return sweep_apply(p, orient, reinterpret_cast<const cplx*>(g), reinterpret_cast<cplx*>(v), false, 1);
}

ls_status ls_bidirectional(ls_plan* p, const double* g, double* v) {
  if (!p || !g || !v || g == v || p->slabs[0].empty()) {
    ls_set_error("ls_bidirectional: bad arguments");
    return LS_EINVAL;
  }
  DeviceGuard dg(p->device);
  if (p->fp32)
    return via_f32(p, g, v, 1, [&](const fcplx* a, fcplx* b) {
      return p->opt.precond == LS_PREC_BD ? inner_prec<fcplx>(p, a, b, 1) : bidirectional_apply(p, a, b, 1);
    });
  const cplx* gi = reinterpret_cast<const cplx*>(g);
  cplx* vo = reinterpret_cast<cplx*>(v);
  return p->opt.precond == LS_PREC_BD ? inner_prec<cplx>(p, gi, vo, 1) : bidirectional_apply(p, gi, vo, 1);
}

ls_status ls_apply_c64(ls_plan* p, const float* v, float* Hv, int batch) {
  if (!p || !v || !Hv || batch < 1 || batch > p->opt.max_batch || !p->fp32) {
    ls_set_error("ls_apply_c64: needs an LS_FP32_REFINE plan and batch in [1, max_batch]");
    return LS_EINVAL;
  }
  DeviceGuard dg(p->device);
  return apply_H32(p, reinterpret_cast<const fcplx*>(v), reinterpret_cast<fcplx*>(Hv), batch, 1.0, 1.0);
}

ls_status ls_sparse_solve(ls_plan* p, const double* g, double* v, int batch, double tol, int max_its,
                          ls_solve_info* info) {
  if (!p || !g || !v || batch < 1 || g == v || !(tol > 0) || max_its < 1) {
    ls_set_error("ls_sparse_solve: bad arguments");
    return LS_EINVAL;
  }
  DeviceGuard dg(p->device);
  const size_t N = (size_t)p->n * p->n;
  bool all = true;
  for (int b0 = 0; b0 < batch; b0 += p->opt.max_batch) {
    const int B = std::min(p->opt.max_batch, batch - b0);
    const auto t0 = std::chrono::steady_clock::now();
    const cplx* gb = reinterpret_cast<const cplx*>(g) + b0 * N;
    cplx* vb = reinterpret_cast<cplx*>(v) + b0 * N;
    std::vector<GmresResult> res;
    auto run = [&](auto tag, const auto* gi, auto* vo) -> ls_status {
      using T = decltype(tag);
      auto op = [&](const T* in, T* out, int nb) { return stencil_apply_C(p, in, out, nb); };
      auto pr = [&](const T* in, T* out, int nb) { return inner_prec<T>(p, in, out, nb); };
      return fgmres<T>(p, op, pr, gi, vo, B, tol, max_its, 0, PK<T>::iV(p), PK<T>::iZ(p), res);
    };
    if (p->fp32) {
      LS_TRY(via_f32(p, g + 2 * b0 * N, v + 2 * b0 * N, B,
                     [&](const fcplx* a, fcplx* o) { return run(fcplx{}, a, o); }));
    } else {
      LS_TRY(run(cplx{}, gb, vb));
    }
    // the recomputed FP64 residual ||g - C v|| / ||g||
    cplx* e = p->vtmp + (size_t)p->opt.max_batch * N;
    std::vector<double> ng(B), ne(B);
    LS_TRY(vec_norms(p, gb, N, B, ng.data()));
    LS_TRY(stencil_residual_C(p, gb, vb, e, B));
    LS_TRY(vec_norms(p, e, N, B, ne.data()));
    LS_HIP(hipStreamSynchronize(p->stream));
    const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    for (int i = 0; i < B; ++i) {
      const double rel = ng[i] > 0 ? ne[i] / ng[i] : 0.0;
      all = all && res[i].converged;
      if (info) {
        ls_solve_info& I = info[b0 + i];
        I.outer_its = res[i].iters;
        I.inner_its_total = 0;
        I.relres_est = res[i].relres;
        I.relres_true = rel;
        I.converged = res[i].converged ? 1 : 0;
        I.t_ms = ms / B;
        I.fno_flags = 0;
      }
    }
  }
  if (!all) {
    ls_set_error("ls_sparse_solve: hit max_its before tol");
    return LS_ENOCONV;
  }
  return LS_OK;
}

ls_status ls_precond_apply(ls_plan* p, const double* r, double* z, int batch) {
  if (!p || !r || !z || batch < 1 || r == z) {
    ls_set_error("ls_precond_apply: bad arguments");
    return LS_EINVAL;
  }
  DeviceGuard dg(p->device);
  const size_t N = (size_t)p->n * p->n;
  bool all = true;
  for (int b0 = 0; b0 < batch; b0 += p->opt.max_batch) {
    const int B = std::min(p->opt.max_batch, batch - b0);
    std::vector<GmresResult> res;
    const double* rb = r + 2 * b0 * N;
    double* zb = z + 2 * b0 * N;
    if (p->fp32) {
      LS_TRY(via_f32(p, rb, zb, B, [&](const fcplx* a, fcplx* o) { return precond_batch<fcplx>(p, a, o, B, res); }));
    } else {
      LS_TRY(precond_batch<cplx>(p, reinterpret_cast<const cplx*>(rb), reinterpret_cast<cplx*>(zb), B, res));
    }
    if (p->opt.inner_fixed_iters == 0)
      for (auto& x : res) all = all && x.converged;
  }
  LS_HIP(hipStreamSynchronize(p->stream));
  if (!all) {
    ls_set_error("ls_precond_apply: inner GMRES hit max_inner");
    return LS_ENOCONV;
  }
  return LS_OK;
}

ls_status ls_solve(ls_plan* p, const double* f, double* u, int batch, double tol,
                   ls_solve_info* info) {
  if (!p || !f || !u || batch < 1 || f == u || !(tol > 0)) {
    ls_set_error("ls_solve: bad arguments");
    return LS_EINVAL;
  }
  DeviceGuard dg(p->device);
  const size_t N = (size_t)p->n * p->n;
  bool all = true;
  for (int b0 = 0; b0 < batch; b0 += p->opt.max_batch) {
    const int B = std::min(p->opt.max_batch, batch - b0);
    const auto t0 = std::chrono::steady_clock::now();
    const cplx* fb = reinterpret_cast<const cplx*>(f) + b0 * N;
    cplx* ub = reinterpret_cast<cplx*>(u) + b0 * N;
    cplx* rbuf = p->vtmp + (size_t)p->opt.max_batch * N;
    std::vector<int> inner_total(B, 0), outer_total(B, 0);
    std::vector<double> nf(B), rel(B, 0.0), est(B, 0.0);
    std::vector<char> conv(B, 0);
    LS_TRY(vec_norms(p, fb, N, B, nf.data()));
    if (!p->fp32) {
      std::vector<GmresResult> res;
      LS_TRY(outer_fgmres<cplx>(p, fb, ub, B, std::vector<double>(B, tol), res, inner_total));
      bool restart = false;
      for (int i = 0; i < B; ++i) {
        outer_total[i] = res[i].iters;
        est[i] = res[i].relres;
      }
      LS_TRY(true_residual(p, fb, ub, rbuf, B, nf, rel));
      // the flag follows the recomputed residual: a right-hand side whose
      // estimate met tol but whose true residual did not is restarted from
      // its iterate (FP64 corrections, at most max_refine)
      for (int i = 0; i < B; ++i) restart = restart || (rel[i] > tol && est[i] <= tol && std::isfinite(rel[i]));
      if (restart) {
        if (!p->solve_buf)
          LS_TRY(plan_alloc(p, (void**)&p->solve_buf, sizeof(cplx) * 2 * (size_t)p->opt.max_batch * N));
        LS_TRY(refine_bd(p, fb, ub, rbuf, p->solve_buf, B, tol, nf, rel, outer_total, inner_total));
      }
      for (int i = 0; i < B; ++i) conv[i] = rel[i] <= tol;
    } else {
      // Iterative refinement: r = f - H u in FP64, d ~ H^{-1} r by FP32
      // flexible GMRES to max(lowp_tol, tol / ||r||_rel), u += d, until
      // ||r|| / ||f|| <= tol for every right-hand side.
      LS_TRY(vec_zero(p, ub, N * B));
      LS_TRY(vec_copy(p, rbuf, fb, N * B));
      for (int i = 0; i < B; ++i) rel[i] = nf[i] > 0 ? 1.0 : 0.0;
      F32Scratch sc;
      LS_TRY(f32_scratch(p, sc));
      for (int it = 0; it < p->opt.max_refine; ++it) {
        bool done = true;
        std::vector<double> scale(B), back(B), tgt(B);
        for (int i = 0; i < B; ++i) {
          const bool act = rel[i] > tol;
          done = done && !act;
          const double nr = rel[i] * nf[i];
          scale[i] = act ? 1.0 / nr : 0.0;   // finished right-hand sides get a zero correction
          back[i] = act ? nr : 0.0;
          tgt[i] = act ? std::max(p->opt.lowp_tol, 0.5 * tol / rel[i]) : 1.0;
        }
        if (done) break;
        LS_TRY(vec_to_f32_b(p, sc.a, rbuf, scale.data(), N, B));
        std::vector<GmresResult> res;
        double tmin = 1.0;
        for (int i = 0; i < B; ++i) if (rel[i] > tol) tmin = std::min(tmin, tgt[i]);
        LS_TRY(outer_fgmres<fcplx>(p, sc.a, sc.b, B, std::vector<double>(B, tmin), res, inner_total));
        for (int i = 0; i < B; ++i) outer_total[i] += (rel[i] > tol) ? res[i].iters : 0;
        LS_TRY(vec_from_f32_b(p, ub, ub, sc.b, back.data(), N, B));
        LS_TRY(true_residual(p, fb, ub, rbuf, B, nf, rel));
      }
      for (int i = 0; i < B; ++i) {
        est[i] = rel[i];
        conv[i] = rel[i] <= tol;
      }
    }
    const auto t1 = std::chrono::steady_clock::now();
    const double ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
    for (int i = 0; i < B; ++i) {
      if (!conv[i]) all = false;
      if (info) {
        ls_solve_info& I = info[b0 + i];
        I.outer_its = outer_total[i];
        I.inner_its_total = inner_total[i];
        I.relres_est = est[i];
        I.relres_true = rel[i];
        I.converged = conv[i] ? 1 : 0;
        I.t_ms = ms / B;
        I.fno_flags = 0;
      }
    }
  }
  LS_HIP(hipStreamSynchronize(p->stream));
  if (!all) {
    ls_set_error("ls_solve: hit max_outer / max_refine before tol");
    return LS_ENOCONV;
  }
  return LS_OK;
}

ls_status ls_solve_multi(ls_plan* const* plans, int count, const double* const* f,
                         double* const* u, const int* batch, double tol,
                         ls_solve_info* const* info) {
  if (!plans || count < 1 || !f || !u || !batch) {
    ls_set_error("ls_solve_multi: bad arguments");
    return LS_EINVAL;
  }
  for (int i = 0; i < count; ++i)
    for (int j = 0; j < i; ++j)
      if (plans[i] == plans[j] || (plans[i] && plans[j] && plans[i]->stream == plans[j]->stream)) {
        ls_set_error("ls_solve_multi: plans must be distinct and use distinct streams");
        return LS_EINVAL;
      }
  std::vector<ls_status> st(count, LS_OK);
  std::vector<std::string> msg(count);
  std::vector<std::thread> th;
  for (int i = 0; i < count; ++i)
    th.emplace_back([&, i]() {
      if (plans[i]) (void)hipSetDevice(plans[i]->device);
      st[i] = ls_solve(plans[i], f[i], u[i], batch[i], tol, info ? info[i] : nullptr);
      msg[i] = g_last_error;
    });
  for (auto& t : th) t.join();
  ls_status worst = LS_OK;
  for (int i = 0; i < count; ++i)
    if (st[i] != LS_OK && (worst == LS_OK || worst == LS_ENOCONV)) {
      worst = st[i];
      g_last_error = "plan " + std::to_string(i) + ": " + msg[i];
    }
  return worst;
}

ls_status ls_solve_fno(ls_plan* p, ls_fno* fn, const double* uI, const double* f, double* u, int batch,
                       double tol, int mode, ls_solve_info* info) {
  if (!p || !fn || !uI || !f || !u || batch < 1 || f == u || !(tol > 0) || mode < 0 ||
      mode > (LS_FNO_WARM | LS_FNO_PREC | LS_FNO_PROBE) ||
      ((mode & LS_FNO_PROBE) && !(mode & LS_FNO_WARM))) {
    ls_set_error("ls_solve_fno: bad arguments");
    return LS_EINVAL;
  }
  if (p->n < 32 || p->n > fno_max_n(fn)) {
    ls_set_error("ls_solve_fno: grid side outside the network's range [32, max_n]");
    return LS_EINVAL;
  }
  DeviceGuard dg(p->device);
  FnoStreamGuard sg(fn, p->stream);
  const int n = p->n;
  const size_t N = (size_t)n * n;
  const size_t BN = (size_t)p->opt.max_batch * N;
  // candidate solution X and its residual R2: FP32 plans have vtmp slots
  // 0 and 2 free (their Alg. 2 runs in vtmp32); FP64 plans get two more
  if (!p->fp32 && !p->solve_buf) LS_TRY(plan_alloc(p, (void**)&p->solve_buf, sizeof(cplx) * 2 * BN));
  cplx* X = p->fp32 ? p->vtmp + 2 * BN : p->solve_buf;
  cplx* R2 = p->fp32 ? p->vtmp : p->solve_buf + BN;
  cplx* rbuf = p->vtmp + BN;
  const int chunk = p->opt.max_batch;  // the network runs in its own sub-batches
  bool all = true;
  // LS_FNO_PROBE: the first right-hand side's warm start decides whether the
  // network is evaluated for the others (same medium, same grid)
  bool probed = !(mode & LS_FNO_PROBE), net_ok = true;
  for (int b0 = 0; b0 < batch; b0 += chunk) {
    const int B = std::min(chunk, batch - b0);
    const auto t0 = std::chrono::steady_clock::now();
    const cplx* fb = reinterpret_cast<const cplx*>(f) + b0 * N;
    const double* uIb = uI + 2 * b0 * N;
    cplx* ub = reinterpret_cast<cplx*>(u) + b0 * N;
    std::vector<int> inner_total(B, 0), outer_total(B, 0), flags(B, 0);
    std::vector<double> nf(B), rel(B, 0.0);
    LS_TRY(vec_norms(p, fb, N, B, nf.data()));
    if (mode & LS_FNO_WARM) {
      int done = 0;  // right-hand sides whose warm start was evaluated
      if (!probed) {
        LS_TRY(fno_residual_map<cplx>(fn, n, 1, p->m, 0, uIb, fb, ub));  // u0 = f + s y
        std::vector<double> rel1;
        LS_TRY(true_residual(p, fb, ub, rbuf, 1, nf, rel1));
        rel[0] = rel1[0];
        net_ok = nf[0] > 0 && rel[0] < 1.0;
        probed = true;
        done = 1;
      }
      if (net_ok && done < B) {
        std::vector<double> nfr(nf.begin() + done, nf.end()), relr;
        LS_TRY(fno_residual_map<cplx>(fn, n, B - done, p->m, 0, uIb + 2 * done * N, fb + done * N,
                                      ub + done * N));
        LS_TRY(true_residual(p, fb + done * N, ub + done * N, rbuf + done * N, B - done, nfr, relr));
        std::copy(relr.begin(), relr.end(), rel.begin() + done);
        done = B;
      }
      for (int i = 0; i < B; ++i) {
        if (i < done && nf[i] > 0 && rel[i] < 1.0) {
          flags[i] |= LS_FNO_WARM_USED;
          continue;
        }
        if (nf[i] > 0) flags[i] |= i < done ? LS_FNO_WARM_REJECTED : LS_FNO_WARM_SKIPPED;
        LS_TRY(vec_zero(p, ub + i * N, N));
        LS_TRY(vec_copy(p, rbuf + i * N, fb + i * N, N));
        rel[i] = nf[i] > 0 ? 1.0 : 0.0;
      }
    } else {
      LS_TRY(vec_zero(p, ub, N * B));
      LS_TRY(vec_copy(p, rbuf, fb, N * B));
      for (int i = 0; i < B; ++i) rel[i] = nf[i] > 0 ? 1.0 : 0.0;
    }
    if ((mode & LS_FNO_PREC) && net_ok) {
      // one flexible-GMRES pass preconditioned by the network; kept per
      // right-hand side only if it at least halves the residual
      std::vector<double> scale, back;
      const double tgt = refine_scales(rel, nf, tol, p->fp32 ? p->opt.lowp_tol : 0.0, scale, back);
      const int maxit = std::max(2, p->opt.max_outer / 4);
      auto net = [&](auto tag) {
        using T = decltype(tag);
        return [&, p](const T* in, T* out, int nb) -> ls_status {
          return fno_residual_map<T>(fn, n, nb, p->m, 0, uIb, in, out);
        };
      };
      std::vector<GmresResult> res;
      LS_TRY(correction(p, rbuf, ub, X, B, scale, back, tgt, maxit, net(cplx{}), net(fcplx{}), res));
      std::vector<double> rel2;
      LS_TRY(true_residual(p, fb, X, R2, B, nf, rel2));
      for (int i = 0; i < B; ++i) {
        if (!(scale[i] > 0)) continue;
        outer_total[i] += res[i].iters;
        if (rel2[i] <= 0.5 * rel[i]) {
          flags[i] |= LS_FNO_PREC_USED;
          LS_TRY(vec_copy(p, ub + i * N, X + i * N, N));
          LS_TRY(vec_copy(p, rbuf + i * N, R2 + i * N, N));
          rel[i] = rel2[i];
        } else {
          flags[i] |= LS_FNO_PREC_FALLBACK;
        }
      }
    }
    LS_TRY(refine_bd(p, fb, ub, rbuf, X, B, tol, nf, rel, outer_total, inner_total));
    LS_HIP(hipStreamSynchronize(p->stream));
    const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    for (int i = 0; i < B; ++i) {
      const bool conv = rel[i] <= tol;
      all = all && conv;
      if (info) {
        ls_solve_info& I = info[b0 + i];
        I.outer_its = outer_total[i];
        I.inner_its_total = inner_total[i];
        I.relres_est = rel[i];
        I.relres_true = rel[i];
        I.converged = conv ? 1 : 0;
        I.t_ms = ms / B;
        I.fno_flags = flags[i];
      }
    }
  }
  if (!all) {
    ls_set_error("ls_solve_fno: hit max_refine before tol");
    return LS_ENOCONV;
  }
  return LS_OK;
}

ls_status ls_solve_fno_multi(ls_plan* const* plans, ls_fno* const* fnos, int count, const double* const* uI,
                             const double* const* f, double* const* u, const int* batch, double tol, int mode,
                             ls_solve_info* const* info) {
  if (!plans || !fnos || count < 1 || !uI || !f || !u || !batch) {
    ls_set_error("ls_solve_fno_multi: bad arguments");
    return LS_EINVAL;
  }
  for (int i = 0; i < count; ++i)
    for (int j = 0; j < i; ++j)
      if (plans[i] == plans[j] || fnos[i] == fnos[j] ||
          (plans[i] && plans[j] && plans[i]->stream == plans[j]->stream)) {
        ls_set_error("ls_solve_fno_multi: plans and networks must be distinct, streams distinct");
        return LS_EINVAL;
      }
  std::vector<ls_status> st(count, LS_OK);
  std::vector<std::string> msg(count);
  std::vector<std::thread> th;
  for (int i = 0; i < count; ++i)
    th.emplace_back([&, i]() {
      if (plans[i]) (void)hipSetDevice(plans[i]->device);
      st[i] = ls_solve_fno(plans[i], fnos[i], uI[i], f[i], u[i], batch[i], tol, mode, info ? info[i] : nullptr);
      msg[i] = g_last_error;
    });
  for (auto& t : th) t.join();
  ls_status worst = LS_OK;
  for (int i = 0; i < count; ++i)
    if (st[i] != LS_OK && (worst == LS_OK || worst == LS_ENOCONV)) {
      worst = st[i];
      g_last_error = "plan " + std::to_string(i) + ": " + msg[i];
    }
  return worst;
}

}  // extern "C"
