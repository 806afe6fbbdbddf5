// Level-1 kernels for the GMRES drivers (Section 4, Alg. 3 and the outer
// loop): multi-vector inner products with a deterministic two-stage
// reduction (always accumulated in FP64), multi-vector updates and linear
// combinations, and the FP64 <-> FP32 conversions of the refinement loop.
// Vectors are complex FP64 or FP32; a set of k vectors has a fixed stride.
#include "ls_internal.h"

#include <algorithm>
#include <vector>

namespace {

constexpr int kDotBlocks = 512;
constexpr int kDotThreads = 256;
constexpr int kGroup = 8;  // vectors per pass over w

template <typename T>
__device__ __forceinline__ cplx up(T a) { return cmk((double)a.x, (double)a.y); }

// partial[b][blk][i] = sum over this block's strided slice of
// conj(V_i[b]) w[b] for right-hand side b = blockIdx.y (V_i[b] at
// V + i*stride + b*N, w[b] at w + b*N), accumulated in FP64 whatever the
// storage precision T.
template <typename T>
__global__ __launch_bounds__(kDotThreads) void k_multidot(const T* __restrict__ V, int k,
                                                          size_t stride,
                                                          const T* __restrict__ w, size_t N,
                                                          cplx* __restrict__ partial) {
  V += (size_t)blockIdx.y * N;
  w += (size_t)blockIdx.y * N;
  partial += (size_t)blockIdx.y * gridDim.x * kGroup;
  cplx acc[kGroup];
#pragma unroll
  for (int i = 0; i < kGroup; ++i) acc[i] = cmk(0, 0);
  for (size_t t = (size_t)blockIdx.x * kDotThreads + threadIdx.x; t < N;
       t += (size_t)gridDim.x * kDotThreads) {
    const cplx wv = up(w[t]);
#pragma unroll
    for (int i = 0; i < kGroup; ++i)
      if (i < k) acc[i] = cfmaconj(up(V[i * stride + t]), wv, acc[i]);
  }
  __shared__ cplx red[kDotThreads];
#pragma unroll
  for (int i = 0; i < kGroup; ++i) {  // constant indices keep acc in registers
    if (i >= k) break;
    red[threadIdx.x] = acc[i];
    __syncthreads();
    for (int s = kDotThreads / 2; s > 0; s >>= 1) {
      if (threadIdx.x < s) red[threadIdx.x] = cadd(red[threadIdx.x], red[threadIdx.x + s]);
      __syncthreads();
    }
    if (threadIdx.x == 0) partial[(size_t)blockIdx.x * kGroup + i] = red[0];
    __syncthreads();
  }
}

// out[b][i] = sum_blk partial[b][blk][i]: one workgroup per (i, b), fixed
// tree order.  out row stride ldo.
__global__ __launch_bounds__(256) void k_finish_dot(const cplx* __restrict__ partial, int nblk,
                                                    cplx* __restrict__ out, int ldo) {
  const int i = blockIdx.x;
  partial += (size_t)blockIdx.y * nblk * kGroup;
  out += (size_t)blockIdx.y * ldo;
  __shared__ cplx red[256];
  cplx s = cmk(0, 0);
  for (int b = threadIdx.x; b < nblk; b += 256) s = cadd(s, partial[(size_t)b * kGroup + i]);
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] = cadd(red[threadIdx.x], red[threadIdx.x + h]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[i] = red[0];
}

// y[b] = y0[b] + sign * sum_i c[b][i] V_i[b] (y0 may be null: 0), in the
// precision of T; b = blockIdx.y, c row stride ldc.
template <typename T>
__global__ void k_multiaxpy(T* __restrict__ y, const T* __restrict__ y0, const T* __restrict__ V,
                            int k, size_t stride, const cplx* __restrict__ c, int ldc, size_t N,
                            double sign) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N) return;
  const size_t off = (size_t)blockIdx.y * N + t;
  c += (size_t)blockIdx.y * ldc;
  T acc = y0 ? y0[off] : tmk<T>(0, 0);
  for (int i = 0; i < k; ++i) acc = tfma(tmk<T>(sign * c[i].x, sign * c[i].y), V[i * stride + off], acc);
  y[off] = acc;
}

// One Gram-Schmidt update fused with the next inner product, for k <=
// kGroup basis vectors: w[b] -= sum_i c[b][i] V_i[b] (c on the device, the
// update in the precision of T exactly as k_multiaxpy forms it), then the
// partial sums of conj(V_i[b]) w[b] (NORM: of |w[b]|^2) exactly as
// k_multidot forms them from the updated w, on the same grid.
template <typename T, bool NORM>
__global__ __launch_bounds__(kDotThreads) void k_update_dot(const T* __restrict__ V, int k, size_t stride,
                                                            T* __restrict__ w, size_t N,
                                                            const cplx* __restrict__ c, int ldc,
                                                            cplx* __restrict__ partial) {
  V += (size_t)blockIdx.y * N;
  w += (size_t)blockIdx.y * N;
  c += (size_t)blockIdx.y * ldc;
  partial += (size_t)blockIdx.y * gridDim.x * kGroup;
  T cf[kGroup];
#pragma unroll
  for (int i = 0; i < kGroup; ++i) cf[i] = i < k ? tmk<T>(-c[i].x, -c[i].y) : tmk<T>(0, 0);
  constexpr int NA = NORM ? 1 : kGroup;
  cplx acc[NA];
#pragma unroll
  for (int i = 0; i < NA; ++i) acc[i] = cmk(0, 0);
  for (size_t t = (size_t)blockIdx.x * kDotThreads + threadIdx.x; t < N;
       t += (size_t)gridDim.x * kDotThreads) {
    T vi[kGroup];
#pragma unroll
    for (int i = 0; i < kGroup; ++i) vi[i] = i < k ? V[i * stride + t] : tmk<T>(0, 0);
    T a = w[t];
#pragma unroll
    for (int i = 0; i < kGroup; ++i)
      if (i < k) a = tfma(cf[i], vi[i], a);
    w[t] = a;
    const cplx wv = up(a);
    if (NORM) {
      acc[0] = cfmaconj(wv, wv, acc[0]);
    } else {
#pragma unroll
      for (int i = 0; i < NA; ++i)
        if (i < k) acc[i] = cfmaconj(up(vi[i]), wv, acc[i]);
    }
  }
  __shared__ cplx red[kDotThreads];
  const int nk = NORM ? 1 : k;
#pragma unroll
  for (int i = 0; i < NA; ++i) {
    if (i >= nk) break;
    red[threadIdx.x] = acc[i];
    __syncthreads();
    for (int s = kDotThreads / 2; s > 0; s >>= 1) {
      if (threadIdx.x < s) red[threadIdx.x] = cadd(red[threadIdx.x], red[threadIdx.x + s]);
      __syncthreads();
    }
    if (threadIdx.x == 0) partial[(size_t)blockIdx.x * kGroup + i] = red[0];
    __syncthreads();
  }
}

// Per-right-hand-side factors, passed by value in the kernel arguments (no
// transfer, nothing for the host to wait on); a launch covers at most
// kScaleChunk right-hand sides.
constexpr int kScaleChunk = 64;
struct Scales {
  double s[kScaleChunk];
};

// y[b] = s[b] * x[b]
template <typename T>
__global__ void k_scale_b(T* __restrict__ y, const T* __restrict__ x, Scales s, size_t N) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N) return;
  const size_t off = (size_t)blockIdx.y * N + t;
  const double f = s.s[blockIdx.y];
  y[off] = tmk<T>(x[off].x * f, x[off].y * f);
}

template <typename T>
__global__ void k_scale_copy(T* __restrict__ y, const T* __restrict__ x, double s, size_t N) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < N) y[t] = tmk<T>(x[t].x * s, x[t].y * s);
}

template <typename T>
__global__ void k_axpy(T* __restrict__ y, const T* __restrict__ x, cplx a, size_t N) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < N) y[t] = tfma(tmk<T>(a.x, a.y), x[t], y[t]);
}

template <typename T>
__global__ void k_fill_zero(T* __restrict__ y, size_t N) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < N) y[t] = tmk<T>(0, 0);
}

// y[b] (FP32) = s[b] * x[b] (FP64)
__global__ void k_down(fcplx* __restrict__ y, const cplx* __restrict__ x, Scales s, size_t N) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N) return;
  const size_t o = (size_t)blockIdx.y * N + t;
  const double f = s.s[blockIdx.y];
  y[o] = make_float2((float)(x[o].x * f), (float)(x[o].y * f));
}

// y[b] (FP64) = y0[b] + s[b] * x[b] (FP32); y0 may be null
__global__ void k_up_axpy(cplx* __restrict__ y, const cplx* __restrict__ y0,
                          const fcplx* __restrict__ x, Scales s, size_t N) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N) return;
  const size_t o = (size_t)blockIdx.y * N + t;
  const double f = s.s[blockIdx.y];
  cplx v = cmk((double)x[o].x * f, (double)x[o].y * f);
  if (y0) v = cadd(y0[o], v);
  y[o] = v;
}

// Reduction partials and the device result / coefficient buffer, with
// pinned host twins for the transfers of the Krylov loop (a pinned copy is
// one DMA, a pageable one is staged through the runtime's own buffer).
ls_status ensure_red(ls_plan* p) {
  if (!p->red) {
    const int B = p->opt.max_batch;
    const size_t small = sizeof(cplx) * 256 * B;
    if (!p->hres) LS_HIP(hipHostMalloc((void**)&p->hres, small, hipHostMallocDefault));
    if (!p->hcoef) LS_HIP(hipHostMalloc((void**)&p->hcoef, small, hipHostMallocDefault));
    if (!p->coef_ev) LS_HIP(hipEventCreateWithFlags(&p->coef_ev, hipEventDisableTiming));
    if (!p->dotbuf) LS_TRY(plan_alloc(p, (void**)&p->dotbuf, small));
    LS_TRY(plan_alloc(p, (void**)&p->red, sizeof(cplx) * kDotBlocks * kGroup * B));
  }
  return LS_OK;
}

inline int blocks_for(size_t N, int t) { return (int)((N + t - 1) / t); }

// Coefficients to the device result buffer through the pinned twin.  The
// host does not wait for the copy: the next upload waits (on the event
// recorded after this copy) before it overwrites the pinned twin.
ls_status upload_coef(ls_plan* p, const cplx* coef_host, size_t cnt) {
  LS_TRY(ensure_red(p));
  if (p->coef_pending) LS_HIP(hipEventSynchronize(p->coef_ev));
  std::copy(coef_host, coef_host + cnt, p->hcoef);
  LS_HIP(hipMemcpyAsync(p->dotbuf, p->hcoef, sizeof(cplx) * cnt, hipMemcpyHostToDevice, p->stream));
  LS_HIP(hipEventRecord(p->coef_ev, p->stream));
  p->coef_pending = true;
  return LS_OK;
}

// The first cnt values of the device result buffer to out_host, through the
// pinned twin; waits for the stream.
ls_status download_results(ls_plan* p, cplx* out_host, size_t cnt) {
  LS_HIP(hipMemcpyAsync(p->hres, p->dotbuf, sizeof(cplx) * cnt, hipMemcpyDeviceToHost, p->stream));
  LS_HIP(hipStreamSynchronize(p->stream));
  p->coef_pending = false;
  std::copy(p->hres, p->hres + cnt, out_host);
  return LS_OK;
}

// Launches fn(c0, cnt, factors) for the right-hand sides c0 .. c0+cnt-1 of
// s_host, kScaleChunk at a time.
template <class F>
ls_status for_scale_chunks(const double* s_host, int B, F fn) {
  for (int c0 = 0; c0 < B; c0 += kScaleChunk) {
    Scales sc{};
    const int cnt = std::min(kScaleChunk, B - c0);
    for (int i = 0; i < cnt; ++i) sc.s[i] = s_host[c0 + i];
    fn(c0, cnt, sc);
  }
  LS_HIP(hipGetLastError());
  return LS_OK;
}

// out_host[b*k + i] = <V_i[b], w[b]> for i < k, b < B.
template <typename T>
ls_status multidot_t(ls_plan* p, const T* V, int k, size_t stride, const T* w, size_t N, int B,
                     cplx* out_host) {
  LS_TRY(ensure_red(p));
  if (k > 256 || B > p->opt.max_batch) {
    ls_set_error("too many Krylov vectors or right-hand sides");
    return LS_EUNSUPPORTED;
  }
  const int nblk = (int)std::min<size_t>(kDotBlocks, (N + kDotThreads - 1) / kDotThreads);
  for (int g0 = 0; g0 < k; g0 += kGroup) {
    const int kk = std::min(kGroup, k - g0);
    k_multidot<T><<<dim3(nblk, B), kDotThreads, 0, p->stream>>>(V + g0 * stride, kk, stride, w, N, p->red);
    k_finish_dot<<<dim3(kk, B), 256, 0, p->stream>>>(p->red, nblk, p->dotbuf + g0, k);
  }
  LS_HIP(hipGetLastError());
  return download_results(p, out_host, (size_t)k * B);
}

template <typename T>
ls_status multiaxpy_t(ls_plan* p, T* y, const T* y0, const T* V, int k, size_t stride,
                      const cplx* coef_host, size_t N, int B, double sign) {
  if (k == 0) {
    if (y0 == nullptr) {
      k_fill_zero<T><<<blocks_for(N * B, 256), 256, 0, p->stream>>>(y, N * B);
      LS_HIP(hipGetLastError());
    }
    return LS_OK;
  }
  LS_TRY(upload_coef(p, coef_host, (size_t)k * B));
  k_multiaxpy<T><<<dim3(blocks_for(N, 256), B), 256, 0, p->stream>>>(y, y0, V, k, stride, p->dotbuf,
                                                                     k, N, sign);
  LS_HIP(hipGetLastError());
  return LS_OK;
}

template <typename T>
ls_status scale_b_t(ls_plan* p, T* y, const T* x, const double* s_host, size_t N, int B) {
  return for_scale_chunks(s_host, B, [&](int c0, int cnt, const Scales& sc) {
    k_scale_b<T><<<dim3(blocks_for(N, 256), cnt), 256, 0, p->stream>>>(y + c0 * N, x + c0 * N, sc, N);
  });
}

// Classical Gram-Schmidt with one re-orthogonalisation of w against the k
// vectors V_i (k <= kGroup): h1 = V^H w, w -= V h1, h2 = V^H w, w -= V h2,
// nrm2 = |w|^2, with each update fused into the next inner product and the
// coefficients kept on the device; one transfer to the host at the end.
// Every value is the one the unfused sequence of multidot / multiaxpy /
// norm calls gives.
template <typename T>
ls_status cgs2_t(ls_plan* p, const T* V, int k, size_t stride, T* w, size_t N, int B, cplx* h1_host,
                 cplx* h2_host, double* nrm2_host) {
  LS_TRY(ensure_red(p));
  if (k < 1 || k > kGroup || B > p->opt.max_batch) {
    ls_set_error("fused Gram-Schmidt step: 1..8 basis vectors");
    return LS_EUNSUPPORTED;
  }
  const int nblk = (int)std::min<size_t>(kDotBlocks, (N + kDotThreads - 1) / kDotThreads);
  cplx* h1 = p->dotbuf;
  cplx* h2 = h1 + (size_t)k * B;
  cplx* nr = h2 + (size_t)k * B;
  k_multidot<T><<<dim3(nblk, B), kDotThreads, 0, p->stream>>>(V, k, stride, w, N, p->red);
  k_finish_dot<<<dim3(k, B), 256, 0, p->stream>>>(p->red, nblk, h1, k);
  k_update_dot<T, false><<<dim3(nblk, B), kDotThreads, 0, p->stream>>>(V, k, stride, w, N, h1, k, p->red);
  k_finish_dot<<<dim3(k, B), 256, 0, p->stream>>>(p->red, nblk, h2, k);
  k_update_dot<T, true><<<dim3(nblk, B), kDotThreads, 0, p->stream>>>(V, k, stride, w, N, h2, k, p->red);
  k_finish_dot<<<dim3(1, B), 256, 0, p->stream>>>(p->red, nblk, nr, 1);
  LS_HIP(hipGetLastError());
  std::vector<cplx> hb((size_t)(2 * k + 1) * B);
  LS_TRY(download_results(p, hb.data(), hb.size()));
  std::copy(hb.begin(), hb.begin() + (size_t)k * B, h1_host);
  std::copy(hb.begin() + (size_t)k * B, hb.begin() + (size_t)2 * k * B, h2_host);
  for (int b = 0; b < B; ++b) nrm2_host[b] = hb[(size_t)2 * k * B + b].x;
  return LS_OK;
}

// partial[b][blk][0] = this block's sum of conj(w[b]) g[b], partial[b][blk][1]
// = of |w[b]|^2 (FP64 accumulation, the layout k_finish_dot reads).
template <typename T>
__global__ __launch_bounds__(kDotThreads) void k_dot_wg(const T* __restrict__ w, const T* __restrict__ g,
                                                        size_t N, cplx* __restrict__ partial) {
  w += (size_t)blockIdx.y * N;
  g += (size_t)blockIdx.y * N;
  partial += (size_t)blockIdx.y * gridDim.x * kGroup;
  cplx acc[2] = {cmk(0, 0), cmk(0, 0)};
  for (size_t t = (size_t)blockIdx.x * kDotThreads + threadIdx.x; t < N;
       t += (size_t)gridDim.x * kDotThreads) {
    const cplx wv = up(w[t]);
    acc[0] = cfmaconj(wv, up(g[t]), acc[0]);
    acc[1] = cfmaconj(wv, wv, acc[1]);
  }
  __shared__ cplx red[kDotThreads];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    red[threadIdx.x] = acc[i];
    __syncthreads();
    for (int s = kDotThreads / 2; s > 0; s >>= 1) {
      if (threadIdx.x < s) red[threadIdx.x] = cadd(red[threadIdx.x], red[threadIdx.x + s]);
      __syncthreads();
    }
    if (threadIdx.x == 0) partial[(size_t)blockIdx.x * kGroup + i] = red[0];
    __syncthreads();
  }
}

// z[b] = alpha_b zt[b], alpha_b = h[b][0] / h[b][1] (0 when h[b][1] = 0; a
// non-finite h[b][1] gives a non-finite z[b]).
template <typename T>
__global__ void k_scale_alpha(T* __restrict__ z, const T* __restrict__ zt, const cplx* __restrict__ h, int ldh,
                              size_t N) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N) return;
  const cplx* hb = h + (size_t)blockIdx.y * ldh;
  const double d = hb[1].x;
  const double ax = d == 0.0 ? 0.0 : hb[0].x / d, ay = d == 0.0 ? 0.0 : hb[0].y / d;
  const size_t off = (size_t)blockIdx.y * N + t;
  z[off] = tmul(tmk<T>(ax, ay), zt[off]);
}

// One step of right-preconditioned GMRES from x0 = 0 in closed form: with zt
// = M g and w = C zt, the one-dimensional minimal-residual solution of
// C x = g over span{zt} is x = alpha zt, alpha = (w^H g) / (w^H w).  Both
// inner products and alpha stay on the device.
template <typename T>
ls_status minres_scale_t(ls_plan* p, const T* w, const T* g, const T* zt, T* z, size_t N, int B) {
  LS_TRY(ensure_red(p));
  if (B > p->opt.max_batch) {
    ls_set_error("one-step inner solve: batch above max_batch");
    return LS_EUNSUPPORTED;
  }
  const int nblk = (int)std::min<size_t>(kDotBlocks, (N + kDotThreads - 1) / kDotThreads);
  cplx* h = p->dotbuf;  // [B][2]
  k_dot_wg<T><<<dim3(nblk, B), kDotThreads, 0, p->stream>>>(w, g, N, p->red);
  k_finish_dot<<<dim3(2, B), 256, 0, p->stream>>>(p->red, nblk, h, 2);
  k_scale_alpha<T><<<dim3(blocks_for(N, 256), B), 256, 0, p->stream>>>(z, zt, h, 2, N);
  LS_HIP(hipGetLastError());
  return LS_OK;
}

}  // namespace

#define LS_BLAS_INSTANCES(T)                                                                     \
  ls_status vec_multidot(ls_plan* p, const T* V, int k, size_t stride, const T* w, size_t N,      \
                         int B, cplx* out_host) {                                                  \
    return multidot_t<T>(p, V, k, stride, w, N, B, out_host);                                      \
  }                                                                                                \
  ls_status vec_multiaxpy(ls_plan* p, T* w, const T* V, int k, size_t stride,                     \
                          const cplx* coef_host, size_t N, int B) {                                \
    return multiaxpy_t<T>(p, w, w, V, k, stride, coef_host, N, B, -1.0);                           \
  }                                                                                                \
  ls_status vec_lincomb(ls_plan* p, T* x, const T* Z, int k, size_t stride,                       \
                        const cplx* coef_host, size_t N, int B) {                                  \
    return multiaxpy_t<T>(p, x, nullptr, Z, k, stride, coef_host, N, B, 1.0);                      \
  }                                                                                                \
  ls_status vec_norms(ls_plan* p, const T* w, size_t N, int B, double* out_host) {                \
    std::vector<cplx> d(B);                                                                        \
    LS_TRY(multidot_t<T>(p, w, 1, 0, w, N, B, d.data()));                                          \
    for (int b = 0; b < B; ++b) /* NaN stays NaN: a poisoned vector must not look converged */     \
      out_host[b] = std::isnan(d[b].x) ? d[b].x : sqrt(fmax(d[b].x, 0.0));                         \
    return LS_OK;                                                                                  \
  }                                                                                                \
  ls_status vec_cgs2(ls_plan* p, const T* V, int k, size_t stride, T* w, size_t N, int B,         \
                     cplx* h1_host, cplx* h2_host, double* nrm2_host) {                            \
    return cgs2_t<T>(p, V, k, stride, w, N, B, h1_host, h2_host, nrm2_host);                       \
  }                                                                                                \
  ls_status vec_minres_scale(ls_plan* p, const T* w, const T* g, const T* zt, T* z, size_t N,      \
                             int B) {                                                              \
    return minres_scale_t<T>(p, w, g, zt, z, N, B);                                                \
  }                                                                                                \
  ls_status vec_norm(ls_plan* p, const T* w, size_t N, double* out_host) {                        \
    return vec_norms(p, w, N, 1, out_host);                                                        \
  }                                                                                                \
  ls_status vec_scale_b(ls_plan* p, T* y, const T* x, const double* s_host, size_t N, int B) {    \
    return scale_b_t<T>(p, y, x, s_host, N, B);                                                    \
  }                                                                                                \
  ls_status vec_scale_copy(ls_plan* p, T* y, const T* x, double s, size_t N) {                    \
    k_scale_copy<T><<<blocks_for(N, 256), 256, 0, p->stream>>>(y, x, s, N);                        \
    LS_HIP(hipGetLastError());                                                                     \
    return LS_OK;                                                                                  \
  }                                                                                                \
  ls_status vec_axpy(ls_plan* p, T* y, const T* x, cplx a, size_t N) {                            \
    k_axpy<T><<<blocks_for(N, 256), 256, 0, p->stream>>>(y, x, a, N);                              \
    LS_HIP(hipGetLastError());                                                                     \
    return LS_OK;                                                                                  \
  }                                                                                                \
  ls_status vec_zero(ls_plan* p, T* y, size_t N) {                                                 \
    k_fill_zero<T><<<blocks_for(N, 256), 256, 0, p->stream>>>(y, N);                               \
    LS_HIP(hipGetLastError());                                                                     \
    return LS_OK;                                                                                  \
  }                                                                                                \
  ls_status vec_copy(ls_plan* p, T* y, const T* x, size_t N) {                                     \
    if (y == x) return LS_OK;                                                                      \
    LS_HIP(hipMemcpyAsync(y, x, N * sizeof(T), hipMemcpyDeviceToDevice, p->stream));               \
    return LS_OK;                                                                                  \
  }

LS_BLAS_INSTANCES(cplx)
LS_BLAS_INSTANCES(fcplx)

ls_status vec_to_f32_b(ls_plan* p, fcplx* y, const cplx* x, const double* s_host, size_t N, int B) {
  return for_scale_chunks(s_host, B, [&](int c0, int cnt, const Scales& sc) {
    k_down<<<dim3(blocks_for(N, 256), cnt), 256, 0, p->stream>>>(y + c0 * N, x + c0 * N, sc, N);
  });
}

ls_status vec_from_f32_b(ls_plan* p, cplx* y, const cplx* y0, const fcplx* x, const double* s_host,
                         size_t N, int B) {
  return for_scale_chunks(s_host, B, [&](int c0, int cnt, const Scales& sc) {
    k_up_axpy<<<dim3(blocks_for(N, 256), cnt), 256, 0, p->stream>>>(
        y + c0 * N, y0 ? y0 + c0 * N : nullptr, x + c0 * N, sc, N);
  });
}

ls_status vec_to_f32(ls_plan* p, fcplx* y, const cplx* x, double s, size_t N) {
  return vec_to_f32_b(p, y, x, &s, N, 1);
}

ls_status vec_from_f32(ls_plan* p, cplx* y, const cplx* y0, const fcplx* x, double s, size_t N) {
  return vec_from_f32_b(p, y, y0, x, &s, N, 1);
}
