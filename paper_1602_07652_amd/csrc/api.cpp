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

ls_status ensure_krylov(ls_plan* p, KrylovSpace& K, int nvec) {
  if (K.cap >= nvec) return LS_OK;
  const size_t N = (size_t)p->n * p->n;
  cplx* nb = nullptr;
  // a larger basis replaces the old one (which stays owned by the plan and
  // is freed with it); bases hold no state across calls
  LS_TRY(plan_alloc(p, (void**)&nb, sizeof(cplx) * N * nvec));
  K.base = nb;
  K.cap = nvec;
  return LS_OK;
}

struct GmresResult {
  int iters = 0;
  double relres = 0.0;
  bool converged = false;
};

// Flexible GMRES: op and prec are callables (in, out) -> ls_status.
template <class Op, class Prec>
ls_status fgmres(ls_plan* p, Op op, Prec prec, const cplx* b, cplx* x, double tol, int maxit,
                 int fixed, KrylovSpace& KV, KrylovSpace& KZ, GmresResult& res) {
  const size_t N = (size_t)p->n * p->n;
  const int limit = fixed > 0 ? fixed : maxit;
  double beta = 0.0;
  LS_TRY(vec_norm(p, b, N, &beta));
  res = GmresResult{};
  if (beta == 0.0) {
    LS_TRY(vec_zero(p, x, N));
    res.converged = true;
    return LS_OK;
  }
  LS_TRY(ensure_krylov(p, KV, limit + 1));
  LS_TRY(ensure_krylov(p, KZ, limit));
  auto V = [&](int i) { return KV.base + (size_t)i * N; };
  auto Z = [&](int i) { return KZ.base + (size_t)i * N; };
  LS_TRY(vec_scale_copy(p, V(0), b, 1.0 / beta, N));
  std::vector<std::vector<zc>> H;  // columns
  std::vector<double> cs;
  std::vector<zc> sn;
  std::vector<zc> gv{zc(beta, 0.0)};
  std::vector<cplx> h1(limit + 1), h2(limit + 1);
  int jdone = 0;
  double rel = 1.0;
  for (int j = 0; j < limit; ++j) {
    LS_TRY(prec(V(j), Z(j)));
    cplx* w = V(j + 1);
    LS_TRY(op(Z(j), w));
    LS_TRY(vec_multidot(p, KV.base, j + 1, N, w, N, h1.data()));
    LS_TRY(vec_multiaxpy(p, w, KV.base, j + 1, N, h1.data(), N));
    LS_TRY(vec_multidot(p, KV.base, j + 1, N, w, N, h2.data()));
    LS_TRY(vec_multiaxpy(p, w, KV.base, j + 1, N, h2.data(), N));
    double hn = 0.0;
    LS_TRY(vec_norm(p, w, N, &hn));
    std::vector<zc> col(j + 2);
    for (int i = 0; i <= j; ++i) col[i] = toz(h1[i]) + toz(h2[i]);
    col[j + 1] = zc(hn, 0.0);
    for (int i = 0; i < j; ++i) {
      const zc a = col[i], bb = col[i + 1];
      col[i] = cs[i] * a + sn[i] * bb;
      col[i + 1] = -std::conj(sn[i]) * a + cs[i] * bb;
    }
    const zc a = col[j];
    const double bb = col[j + 1].real();
    const double r = std::hypot(std::abs(a), bb);
    double c;
    zc s;
    if (std::abs(a) == 0.0) {
      c = 0.0;
      s = zc(1.0, 0.0);
      col[j] = zc(bb, 0.0);
    } else {
      const zc ph = a / std::abs(a);
      c = std::abs(a) / r;
      s = ph * bb / r;
      col[j] = ph * r;
    }
    col[j + 1] = 0.0;
    cs.push_back(c);
    sn.push_back(s);
    gv.push_back(-std::conj(s) * gv[j]);
    gv[j] = c * gv[j];
    H.push_back(col);
    rel = std::abs(gv[j + 1]) / beta;
    jdone = j + 1;
    const bool done = (fixed == 0 && rel <= tol) || rel <= 1e-15 || hn == 0.0;
    if (done || j + 1 == limit) break;
    LS_TRY(vec_scale_copy(p, V(j + 1), w, 1.0 / hn, N));
  }
  // R y = g
  std::vector<zc> y(jdone);
  for (int i = jdone - 1; i >= 0; --i) {
    zc s = gv[i];
    for (int k = i + 1; k < jdone; ++k) s -= H[k][i] * y[k];
    y[i] = s / H[i][i];
  }
  std::vector<cplx> yc(jdone);
  for (int i = 0; i < jdone; ++i) yc[i] = fromz(y[i]);
  LS_TRY(vec_lincomb(p, x, KZ.base, jdone, N, yc.data(), N));
  res.iters = jdone;
  res.relres = rel;
  res.converged = rel <= tol;
  return LS_OK;
}

ls_status inner_prec(ls_plan* p, const cplx* in, cplx* out) {
  const size_t N = (size_t)p->n * p->n;
  switch (p->opt.precond) {
    case LS_PREC_BD:
      return bidirectional_apply(p, in, out);
    case LS_PREC_PT1:
      return sweep_apply(p, 0, in, out, false);
    default:
      return vec_copy(p, out, in, N);
  }
}

// Alg. 3 for one right-hand side.
ls_status precond_one(ls_plan* p, const cplx* r, cplx* z, GmresResult& res) {
  const size_t N = (size_t)p->n * p->n;
  if (!p->inner_rhs) LS_TRY(plan_alloc(p, (void**)&p->inner_rhs, sizeof(cplx) * N));
  LS_TRY(stencil_apply_A(p, r, p->inner_rhs, 1));
  auto op = [&](const cplx* in, cplx* out) { return stencil_apply_C(p, in, out, 1); };
  auto pr = [&](const cplx* in, cplx* out) { return inner_prec(p, in, out); };
  return fgmres(p, op, pr, p->inner_rhs, z, p->opt.inner_tol, p->opt.max_inner,
                p->opt.inner_fixed_iters, p->innerV, p->innerZ, res);
}

bool valid_opts(const ls_options& o) {
  return o.ext >= 0 && o.inner_tol > 0 && o.max_outer >= 1 && o.max_inner >= 1 &&
         o.precision == LS_FP64 && o.precond >= LS_PREC_BD && o.precond <= LS_PREC_NONE &&
         o.inner_fixed_iters >= 0 && o.max_batch >= 1 && o.slabs >= 0 && std::isfinite(o.shift_c);
}

}  // namespace

void ls_set_error(const std::string& msg) { g_last_error = msg; }

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
  for (void* a : p->allocs) (void)hipFree(a);
  delete p;
  return LS_OK;
}

static ls_status create_impl(ls_plan* p, const double* m) {
  const int n = p->n;
  LS_TRY(plan_alloc(p, (void**)&p->m, sizeof(double) * n * n));
  LS_HIP(hipMemcpyAsync(p->m, m, sizeof(double) * n * n, hipMemcpyDeviceToDevice, p->stream));
  LS_TRY(fft_setup_twiddles(p));
  LS_TRY(plan_alloc(p, (void**)&p->stencil_d, sizeof(cplx) * 324));
  LS_TRY(plan_alloc(p, (void**)&p->spec, sizeof(cplx) * p->spec_side * p->spec_side));
  {
    cplx* circ = nullptr;
    LS_HIP(hipMalloc(&circ, sizeof(cplx) * (size_t)p->P * p->P));
    ls_status s = launch_circulant(p, circ);
    if (s == LS_OK) s = stencils_build(p, circ);
    if (s == LS_OK) s = fft2_full_forward(p, circ);
    if (s == LS_OK) s = spectrum_extract(p, circ);
    if (s == LS_OK && hipStreamSynchronize(p->stream) != hipSuccess) s = LS_EDEVICE;
    (void)hipFree(circ);
    if (s != LS_OK) return s;
  }
  LS_TRY(plan_alloc(p, (void**)&p->fft_work, sizeof(cplx) * (size_t)p->opt.max_batch * n * p->P));
  LS_TRY(plan_alloc(p, (void**)&p->vtmp, sizeof(cplx) * (size_t)3 * n * n));
  if (p->opt.precond != LS_PREC_NONE) LS_TRY(slabs_build(p));
  LS_HIP(hipStreamSynchronize(p->stream));
  return LS_OK;
}

ls_status ls_plan_create(ls_plan** out, int n, double h, double omega, const double* m,
                         const ls_options* opt, void* stream) {
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
  ls_status s = create_impl(p, m);
  if (s != LS_OK) {
    std::string keep = g_last_error;
    ls_plan_destroy(p);
    g_last_error = keep;
    return s;
  }
  *out = p;
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
  LS_TRY(vec_copy(p, reinterpret_cast<cplx*>(x), reinterpret_cast<const cplx*>(b),
                  (size_t)p->n * s.q));
  return slab_solve_frame(p, s, reinterpret_cast<cplx*>(x));
}

ls_status ls_sweep(ls_plan* p, int orient, const double* g, double* v) {
  if (!p || !g || !v || g == v || orient < 0 || orient > 1 || p->slabs[orient].empty()) {
    ls_set_error("ls_sweep: bad arguments");
    return LS_EINVAL;
  }
  DeviceGuard dg(p->device);
  return sweep_apply(p, orient, reinterpret_cast<const cplx*>(g), reinterpret_cast<cplx*>(v), false);
}

ls_status ls_bidirectional(ls_plan* p, const double* g, double* v) {
  if (!p || !g || !v || g == v || p->slabs[0].empty()) {
    ls_set_error("ls_bidirectional: bad arguments");
    return LS_EINVAL;
  }
  DeviceGuard dg(p->device);
  return bidirectional_apply(p, reinterpret_cast<const cplx*>(g), reinterpret_cast<cplx*>(v));
}

ls_status ls_precond_apply(ls_plan* p, const double* r, double* z, int batch) {
  if (!p || !r || !z || batch < 1 || r == z) {
    ls_set_error("ls_precond_apply: bad arguments");
    return LS_EINVAL;
  }
  DeviceGuard dg(p->device);
  const size_t N = (size_t)p->n * p->n;
  bool all = true;
  for (int b = 0; b < batch; ++b) {
    GmresResult res;
    LS_TRY(precond_one(p, reinterpret_cast<const cplx*>(r) + b * N,
                       reinterpret_cast<cplx*>(z) + b * N, res));
    if (p->opt.inner_fixed_iters == 0 && !res.converged) all = false;
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
  for (int b = 0; b < batch; ++b) {
    const auto t0 = std::chrono::steady_clock::now();
    const cplx* fb = reinterpret_cast<const cplx*>(f) + b * N;
    cplx* ub = reinterpret_cast<cplx*>(u) + b * N;
    int inner_total = 0;
    auto op = [&](const cplx* in, cplx* out) { return apply_H(p, in, out, 1, 1.0, 1.0); };
    auto pr = [&](const cplx* in, cplx* out) -> ls_status {
      GmresResult r;
      ls_status s = precond_one(p, in, out, r);
      inner_total += r.iters;
      return s;
    };
    GmresResult res;
    LS_TRY(fgmres(p, op, pr, fb, ub, tol, p->opt.max_outer, 0, p->outerV, p->outerZ, res));
    // true residual ||f - H u|| / ||f||
    double nf = 0.0, nr = 0.0;
    cplx* rbuf = p->vtmp + N;
    LS_TRY(apply_H(p, ub, rbuf, 1, 1.0, 1.0));
    LS_TRY(vec_axpy(p, rbuf, fb, cmk(-1.0, 0.0), N));
    LS_TRY(vec_norm(p, rbuf, N, &nr));
    LS_TRY(vec_norm(p, fb, N, &nf));
    const auto t1 = std::chrono::steady_clock::now();
    if (!res.converged) all = false;
    if (info) {
      info[b].outer_its = res.iters;
      info[b].inner_its_total = inner_total;
      info[b].relres_est = res.relres;
      info[b].relres_true = nf > 0 ? nr / nf : 0.0;
      info[b].converged = res.converged ? 1 : 0;
      info[b].t_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
    }
  }
  LS_HIP(hipStreamSynchronize(p->stream));
  if (!all) {
    ls_set_error("ls_solve: outer flexible GMRES hit max_outer");
    return LS_ENOCONV;
  }
  return LS_OK;
}

}  // extern "C"
