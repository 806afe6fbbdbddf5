// Level-1 kernels for the GMRES drivers (Section 4, Alg. 3 and the outer
// loop): multi-vector inner products with a deterministic two-stage
// reduction, multi-vector updates and linear combinations.  Vectors are
// complex FP64; a set of k vectors is stored with a fixed stride.
#include "ls_internal.h"

#include <vector>

namespace {

constexpr int kDotBlocks = 512;
constexpr int kDotThreads = 256;
constexpr int kGroup = 8;  // vectors per pass over w

// partial[blk][i] = sum over this block's strided slice of conj(V_i) w
__global__ __launch_bounds__(kDotThreads) void k_multidot(const cplx* __restrict__ V, int k,
                                                          size_t stride,
                                                          const cplx* __restrict__ w, size_t N,
                                                          cplx* __restrict__ partial) {
  cplx acc[kGroup];
#pragma unroll
  for (int i = 0; i < kGroup; ++i) acc[i] = cmk(0, 0);
  for (size_t t = (size_t)blockIdx.x * kDotThreads + threadIdx.x; t < N;
       t += (size_t)gridDim.x * kDotThreads) {
    const cplx wv = w[t];
#pragma unroll
    for (int i = 0; i < kGroup; ++i)
      if (i < k) acc[i] = cfmaconj(V[i * stride + t], wv, acc[i]);
  }
  __shared__ cplx red[kDotThreads];
  for (int i = 0; i < k; ++i) {
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

__global__ void k_finish_dot(const cplx* __restrict__ partial, int nblk, int k,
                             cplx* __restrict__ out) {
  const int i = threadIdx.x;
  if (i >= k) return;
  cplx s = cmk(0, 0);
  for (int b = 0; b < nblk; ++b) s = cadd(s, partial[(size_t)b * kGroup + i]);
  out[i] = s;
}

// y = y0 - sum_i c_i V_i  (sign = -1) or y = y0 + sum (sign = +1); y0 may
// be null (treated as 0).
__global__ void k_multiaxpy(cplx* __restrict__ y, const cplx* __restrict__ y0,
                            const cplx* __restrict__ V, int k, size_t stride,
                            const cplx* __restrict__ c, size_t N, double sign) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N) return;
  cplx acc = y0 ? y0[t] : cmk(0, 0);
  for (int i = 0; i < k; ++i) {
    const cplx ci = cscale(c[i], sign);
    acc = cfma(ci, V[i * stride + t], acc);
  }
  y[t] = acc;
}

__global__ void k_scale_copy(cplx* __restrict__ y, const cplx* __restrict__ x, double s, size_t N) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < N) y[t] = cscale(x[t], s);
}

__global__ void k_axpy(cplx* __restrict__ y, const cplx* __restrict__ x, cplx a, size_t N) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < N) y[t] = cfma(a, x[t], y[t]);
}

__global__ void k_fill_zero(cplx* __restrict__ y, size_t N) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < N) y[t] = cmk(0, 0);
}

ls_status ensure_red(ls_plan* p) {
  if (!p->red) {
    LS_TRY(plan_alloc(p, (void**)&p->red, sizeof(cplx) * kDotBlocks * kGroup));
    LS_TRY(plan_alloc(p, (void**)&p->dotbuf, sizeof(cplx) * 256));
  }
  return LS_OK;
}

inline int blocks_for(size_t N, int t) { return (int)((N + t - 1) / t); }

}  // namespace

ls_status vec_multidot(ls_plan* p, const cplx* V, int k, size_t stride, const cplx* w, size_t N,
                       cplx* out_host) {
  LS_TRY(ensure_red(p));
  if (k > 256) {
    ls_set_error("too many Krylov vectors");
    return LS_EUNSUPPORTED;
  }
  const int nblk = (int)std::min<size_t>(kDotBlocks, (N + kDotThreads - 1) / kDotThreads);
  for (int g0 = 0; g0 < k; g0 += kGroup) {
    const int kk = std::min(kGroup, k - g0);
    k_multidot<<<nblk, kDotThreads, 0, p->stream>>>(V + g0 * stride, kk, stride, w, N, p->red);
    k_finish_dot<<<1, 64, 0, p->stream>>>(p->red, nblk, kk, p->dotbuf + g0);
  }
  LS_HIP(hipGetLastError());
  LS_HIP(hipMemcpyAsync(out_host, p->dotbuf, sizeof(cplx) * k, hipMemcpyDeviceToHost, p->stream));
  LS_HIP(hipStreamSynchronize(p->stream));
  return LS_OK;
}

static ls_status upload_coef(ls_plan* p, const cplx* coef_host, int k) {
  LS_TRY(ensure_red(p));
  LS_HIP(hipMemcpyAsync(p->dotbuf, coef_host, sizeof(cplx) * k, hipMemcpyHostToDevice, p->stream));
  return LS_OK;
}

ls_status vec_multiaxpy(ls_plan* p, cplx* w, const cplx* V, int k, size_t stride,
                        const cplx* coef_host, size_t N) {
  if (k == 0) return LS_OK;
  LS_TRY(upload_coef(p, coef_host, k));
  k_multiaxpy<<<blocks_for(N, 256), 256, 0, p->stream>>>(w, w, V, k, stride, p->dotbuf, N, -1.0);
  LS_HIP(hipGetLastError());
  // the coefficient buffer is reused by the next call
  LS_HIP(hipStreamSynchronize(p->stream));
  return LS_OK;
}

ls_status vec_lincomb(ls_plan* p, cplx* x, const cplx* Z, int k, size_t stride,
                      const cplx* coef_host, size_t N) {
  LS_TRY(upload_coef(p, coef_host, k));
  k_multiaxpy<<<blocks_for(N, 256), 256, 0, p->stream>>>(x, nullptr, Z, k, stride, p->dotbuf, N, 1.0);
  LS_HIP(hipGetLastError());
  LS_HIP(hipStreamSynchronize(p->stream));
  return LS_OK;
}

ls_status vec_norm(ls_plan* p, const cplx* w, size_t N, double* out_host) {
  cplx d;
  LS_TRY(vec_multidot(p, w, 1, 0, w, N, &d));
  *out_host = sqrt(fmax(d.x, 0.0));
  return LS_OK;
}

ls_status vec_scale_copy(ls_plan* p, cplx* y, const cplx* x, double s, size_t N) {
  k_scale_copy<<<blocks_for(N, 256), 256, 0, p->stream>>>(y, x, s, N);
  LS_HIP(hipGetLastError());
  return LS_OK;
}

ls_status vec_axpy(ls_plan* p, cplx* y, const cplx* x, cplx a, size_t N) {
  k_axpy<<<blocks_for(N, 256), 256, 0, p->stream>>>(y, x, a, N);
  LS_HIP(hipGetLastError());
  return LS_OK;
}

ls_status vec_zero(ls_plan* p, cplx* y, size_t N) {
  k_fill_zero<<<blocks_for(N, 256), 256, 0, p->stream>>>(y, N);
  LS_HIP(hipGetLastError());
  return LS_OK;
}

ls_status vec_copy(ls_plan* p, cplx* y, const cplx* x, size_t N) {
  if (y == x) return LS_OK;
  LS_HIP(hipMemcpyAsync(y, x, N * sizeof(cplx), hipMemcpyDeviceToDevice, p->stream));
  return LS_OK;
}
