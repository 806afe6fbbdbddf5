// Sparsifying stencils and the sparse operators A and C.
//
// Section 2: A has the pattern of the 9-point neighbourhood mu(k); its
// stencil alpha minimises ||alpha G(mu(0), mu(0)^c)|| over unit vectors,
// i.e. alpha is the conjugate of the left singular vector of the smallest
// singular value of M = G(mu, mu^c).  Section 4.1: this is the SVD of a
// 9 x N matrix.  Here M M^* (|mu| x |mu|, Hermitian) is formed by a
// deterministic FP64 reduction over the grid, and its smallest eigenvector
// is found with cyclic Jacobi on the equivalent real symmetric matrix
// [[Re, -Im], [Im, Re]].  Boundary points use the same minimisation with
// mu clipped to the grid (types: low edge / interior / high edge per
// axis), with representative points at the grid centre, edge midpoints and
// corners.  The phase is fixed so that the centre coefficient is real and
// positive.  C = A H on A's pattern: C(k, k+d) = alpha_d + omega^2 beta_d
// m_{k+d}, beta_d = sum_{d'} alpha_{d'} w_{d'-d} (Section 2).
//
// Stencil tables: index ((tz*3 + tx)*3 + dz+1)*3 + dx+1.
#include "ls_internal.h"

#include <cmath>

namespace {

__device__ __forceinline__ void type_range(int t, int& lo, int& hi) {
  lo = (t == 0) ? 0 : -1;
  hi = (t == 2) ? 0 : 1;
}

__device__ __forceinline__ int type_rep(int t, int n) { return t == 0 ? 0 : (t == 1 ? n / 2 : n - 1); }

__device__ __forceinline__ cplx wq(const cplx* __restrict__ circ, int P, int qx, int qz) {
  const int x = qx < 0 ? qx + P : qx;
  const int z = qz < 0 ? qz + P : qz;
  return circ[(size_t)z * P + x];
}

// One workgroup per (type, d, d'), d <= d' in the type's offset list:
// gram[type][d][d'] = sum_{p not in mu(k0)} w_{k0+d-p} conj(w_{k0+d'-p}).
__global__ __launch_bounds__(256) void k_gram(const cplx* __restrict__ circ, int n, int P,
                                              cplx* __restrict__ gram) {
  const int type = blockIdx.y;
  const int tz = type / 3, tx = type % 3;
  int zlo, zhi, xlo, xhi;
  type_range(tz, zlo, zhi);
  type_range(tx, xlo, xhi);
  const int nx = xhi - xlo + 1, nz = zhi - zlo + 1, mt = nx * nz;
  const int pair = blockIdx.x;  // d1 * 9 + d2
  const int d1 = pair / 9, d2 = pair % 9;
  if (d1 >= mt || d2 >= mt || d2 < d1) return;
  const int dz1 = zlo + d1 / nx, dx1 = xlo + d1 % nx;
  const int dz2 = zlo + d2 / nx, dx2 = xlo + d2 % nx;
  const int j0 = type_rep(tz, n), i0 = type_rep(tx, n);
  cplx acc = cmk(0.0, 0.0);
  const int N = n * n;
  for (int k = threadIdx.x; k < N; k += blockDim.x) {
    const int pj = k / n, pi = k % n;
    const int ddz = pj - j0, ddx = pi - i0;
    if (ddz >= zlo && ddz <= zhi && ddx >= xlo && ddx <= xhi) continue;  // p in mu(k0)
    const cplx a = wq(circ, P, i0 + dx1 - pi, j0 + dz1 - pj);
    const cplx b = wq(circ, P, i0 + dx2 - pi, j0 + dz2 - pj);
    acc = cfmaconj(b, a, acc);  // a * conj(b)
  }
  __shared__ double sre[256], sim[256];
  sre[threadIdx.x] = acc.x;
  sim[threadIdx.x] = acc.y;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      sre[threadIdx.x] += sre[threadIdx.x + s];
      sim[threadIdx.x] += sim[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    gram[type * 81 + d1 * 9 + d2] = cmk(sre[0], sim[0]);
    gram[type * 81 + d2 * 9 + d1] = cmk(sre[0], -sim[0]);
  }
}

// One thread per type: smallest eigenvector of the Gram matrix, phase fix,
// then beta.  Writes alpha/beta tables (81 each) and their transposes.
__global__ void k_stencil_solve(const cplx* __restrict__ gram, const cplx* __restrict__ circ,
                                int P, cplx* __restrict__ tables, int* __restrict__ status) {
  const int type = threadIdx.x;
  if (type >= 9) return;
  const int tz = type / 3, tx = type % 3;
  int zlo, zhi, xlo, xhi;
  type_range(tz, zlo, zhi);
  type_range(tx, xlo, xhi);
  const int nx = xhi - xlo + 1, nz = zhi - zlo + 1, mt = nx * nz, M = 2 * mt;
  double A[18][18], V[18][18];
  for (int r = 0; r < M; ++r)
    for (int c = 0; c < M; ++c) V[r][c] = (r == c) ? 1.0 : 0.0;
  for (int r = 0; r < mt; ++r)
    for (int c = 0; c < mt; ++c) {
      const cplx g = gram[type * 81 + r * 9 + c];
      A[r][c] = g.x;
      A[r + mt][c + mt] = g.x;
      A[r][c + mt] = -g.y;
      A[r + mt][c] = g.y;
    }
  double scale = 0.0;
  for (int r = 0; r < M; ++r) scale = fmax(scale, fabs(A[r][r]));
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0;
    for (int p = 0; p < M; ++p)
      for (int q = p + 1; q < M; ++q) off += A[p][q] * A[p][q];
    if (off <= 1e-36 * scale * scale) break;
    for (int p = 0; p < M; ++p)
      for (int q = p + 1; q < M; ++q) {
        const double apq = A[p][q];
        if (fabs(apq) <= 1e-300) continue;
        const double theta = (A[q][q] - A[p][p]) / (2.0 * apq);
        const double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
        const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < M; ++k) {
          const double akp = A[k][p], akq = A[k][q];
          A[k][p] = c * akp - s * akq;
          A[k][q] = s * akp + c * akq;
        }
        for (int k = 0; k < M; ++k) {
          const double apk = A[p][k], aqk = A[q][k];
          A[p][k] = c * apk - s * aqk;
          A[q][k] = s * apk + c * aqk;
        }
        for (int k = 0; k < M; ++k) {
          const double vkp = V[k][p], vkq = V[k][q];
          V[k][p] = c * vkp - s * vkq;
          V[k][q] = s * vkp + c * vkq;
        }
      }
  }
  int imin = 0;
  for (int r = 1; r < M; ++r)
    if (A[r][r] < A[imin][imin]) imin = r;
  // complex eigenvector u = x + i y; alpha = conj(u), phase-fixed.
  cplx al[9];
  double nrm = 0.0;
  for (int r = 0; r < mt; ++r) {
    al[r] = cmk(V[r][imin], -V[r + mt][imin]);
    nrm += al[r].x * al[r].x + al[r].y * al[r].y;
  }
  nrm = sqrt(nrm);
  const int centre = (0 - zlo) * nx + (0 - xlo);
  const cplx cc = al[centre];
  const double ac = sqrt(cc.x * cc.x + cc.y * cc.y);
  if (!(ac > 0.0) || !(nrm > 0.0)) {
    atomicOr(status, 1);
    return;
  }
  const cplx ph = cmk(cc.x / ac / nrm, -cc.y / ac / nrm);  // conj(cc)/|cc| / nrm
  for (int r = 0; r < mt; ++r) al[r] = cmul(al[r], ph);
  al[centre].y = 0.0;
  cplx* alpha = tables;
  cplx* beta = tables + 81;
  cplx* alphaT = tables + 162;
  cplx* betaT = tables + 243;
  const int typeT = tx * 3 + tz;
  for (int e = 0; e < 9; ++e) {
    alpha[type * 9 + e] = cmk(0.0, 0.0);
    beta[type * 9 + e] = cmk(0.0, 0.0);
    alphaT[typeT * 9 + e] = cmk(0.0, 0.0);
    betaT[typeT * 9 + e] = cmk(0.0, 0.0);
  }
  for (int d = 0; d < mt; ++d) {
    const int dz = zlo + d / nx, dx = xlo + d % nx;
    cplx b = cmk(0.0, 0.0);
    for (int e = 0; e < mt; ++e) {
      const int ez = zlo + e / nx, ex = xlo + e % nx;
      b = cfma(al[e], wq(circ, P, ex - dx, ez - dz), b);
    }
    const int slot = (dz + 1) * 3 + (dx + 1);
    const int slotT = (dx + 1) * 3 + (dz + 1);
    alpha[type * 9 + slot] = al[d];
    beta[type * 9 + slot] = b;
    alphaT[typeT * 9 + slotT] = al[d];
    betaT[typeT * 9 + slotT] = b;
  }
}

__device__ __forceinline__ int axis_type(int i, int n) { return i == 0 ? 0 : (i == n - 1 ? 2 : 1); }

// y = A r (mode 0), y = C v (mode 1), y = g - C v (mode 2); T = double2
// or float2 (tables and arithmetic in that precision).  Thread i takes
// column i of RW consecutive rows: a window of three rows of in (and m) at
// columns i - 1, i, i + 1 rolls down the rows, so each input is loaded
// three times (neighbouring lanes, mostly cache hits) instead of nine; the
// interior point type's coefficients are loaded once (uniform addresses),
// the boundary types' per point.  Values outside the grid enter as zeros,
// which leaves every sum as the tap-by-tap sum over the grid points.
template <typename T, typename R, int MODE, int RW>
__global__ __launch_bounds__(128) void k_stencil(const T* __restrict__ in, const T* __restrict__ g,
                                                 T* __restrict__ out, const T* __restrict__ tables,
                                                 const R* __restrict__ m, int n, R omega2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j0 = blockIdx.y * RW;
  const size_t base = (size_t)blockIdx.z * n * n;
  if (i >= n) return;
  const int ti = axis_type(i, n);
  T ai[9], bi[9];
#pragma unroll
  for (int s = 0; s < 9; ++s) {
    ai[s] = tables[4 * 9 + s];
    bi[s] = tables[81 + 4 * 9 + s];
  }
  T v[3][3];
  R mw[3][3];
#pragma unroll
  for (int w = 0; w < 2; ++w) {  // rows j0 - 1 and j0
    const int jj = j0 - 1 + w;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const int ii = i + d - 1;
      const bool ok = jj >= 0 && jj < n && ii >= 0 && ii < n;
      const size_t idx = ok ? (size_t)jj * n + ii : 0;
      v[w + 1][d] = ok ? in[base + idx] : tmk<T>(0, 0);
      mw[w + 1][d] = (MODE != 0 && ok) ? m[idx] : (R)0;
    }
  }
#pragma unroll
  for (int r = 0; r < RW; ++r) {
    const int j = j0 + r;
#pragma unroll
    for (int d = 0; d < 3; ++d) {  // roll the window down one row
      v[0][d] = v[1][d];
      v[1][d] = v[2][d];
      mw[0][d] = mw[1][d];
      mw[1][d] = mw[2][d];
      const int jj = j + 1, ii = i + d - 1;
      const bool ok = jj < n && ii >= 0 && ii < n;
      const size_t idx = ok ? (size_t)jj * n + ii : 0;
      v[2][d] = ok ? in[base + idx] : tmk<T>(0, 0);
      mw[2][d] = (MODE != 0 && ok) ? m[idx] : (R)0;
    }
    if (j >= n) break;
    const int t = axis_type(j, n) * 3 + ti;
    T acc = tmk<T>(0, 0);
#pragma unroll
    for (int s = 0; s < 9; ++s) {
      T c = t == 4 ? ai[s] : tables[t * 9 + s];
      if (MODE != 0) {
        const T b = t == 4 ? bi[s] : tables[81 + t * 9 + s];
        const R f = omega2 * mw[s / 3][s % 3];
        c.x = fma(b.x, f, c.x);
        c.y = fma(b.y, f, c.y);
      }
      acc = tfma(c, v[s / 3][s % 3], acc);
    }
    const size_t o = base + (size_t)j * n + i;
    out[o] = (MODE == 2) ? tsub(g[o], acc) : acc;
  }
}

__global__ void k_to_f32(const cplx* __restrict__ a, fcplx* __restrict__ b, int cnt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < cnt) b[i] = make_float2((float)a[i].x, (float)a[i].y);
}

}  // namespace

ls_status stencils_build(ls_plan* p, const cplx* circ) {
  cplx* gram = nullptr;
  int* status = nullptr;
  LS_HIP(hipMalloc(&gram, sizeof(cplx) * 9 * 81));
  LS_HIP(hipMalloc(&status, sizeof(int)));
  LS_HIP(hipMemsetAsync(gram, 0, sizeof(cplx) * 9 * 81, p->stream));
  LS_HIP(hipMemsetAsync(status, 0, sizeof(int), p->stream));
  k_gram<<<dim3(81, 9), 256, 0, p->stream>>>(circ, p->n, p->P, gram);
  LS_HIP(hipGetLastError());
  k_stencil_solve<<<1, 64, 0, p->stream>>>(gram, circ, p->P, p->stencil_d, status);
  LS_HIP(hipGetLastError());
  int st = 0;
  LS_HIP(hipMemcpyAsync(&st, status, sizeof(int), hipMemcpyDeviceToHost, p->stream));
  LS_HIP(hipMemcpyAsync(p->alpha_h, p->stencil_d, sizeof(cplx) * 81, hipMemcpyDeviceToHost, p->stream));
  LS_HIP(hipMemcpyAsync(p->beta_h, p->stencil_d + 81, sizeof(cplx) * 81, hipMemcpyDeviceToHost, p->stream));
  LS_HIP(hipStreamSynchronize(p->stream));
  LS_HIP(hipFree(gram));
  LS_HIP(hipFree(status));
  if (st != 0) {
    ls_set_error("stencil construction: degenerate singular vector");
    return LS_ESINGULAR;
  }
  return LS_OK;
}

template <typename T, typename R>
static ls_status launch_stencil(ls_plan* p, const T* tables, const R* m, int mode, const T* in,
                                const T* g, T* out, int batch) {
  const int n = p->n;
  constexpr int RW = 8;  // rows per thread
  dim3 grid((n + 127) / 128, (n + RW - 1) / RW, batch);
  const R w2 = (R)(p->omega * p->omega);
  if (mode == 0)
    k_stencil<T, R, 0, RW><<<grid, 128, 0, p->stream>>>(in, g, out, tables, m, n, w2);
  else if (mode == 1)
    k_stencil<T, R, 1, RW><<<grid, 128, 0, p->stream>>>(in, g, out, tables, m, n, w2);
  else
    k_stencil<T, R, 2, RW><<<grid, 128, 0, p->stream>>>(in, g, out, tables, m, n, w2);
  LS_HIP(hipGetLastError());
  return LS_OK;
}

ls_status stencils_to_f32(ls_plan* p) {
  k_to_f32<<<2, 256, 0, p->stream>>>(p->stencil_d, p->f32.stencil, 324);
  LS_HIP(hipGetLastError());
  return LS_OK;
}

ls_status stencil_apply_A(ls_plan* p, const cplx* r, cplx* y, int batch) {
  return launch_stencil<cplx, double>(p, p->stencil_d, p->m, 0, r, nullptr, y, batch);
}
ls_status stencil_apply_C(ls_plan* p, const cplx* v, cplx* y, int batch) {
  return launch_stencil<cplx, double>(p, p->stencil_d, p->m, 1, v, nullptr, y, batch);
}
ls_status stencil_residual_C(ls_plan* p, const cplx* g, const cplx* u, cplx* e, int batch) {
  return launch_stencil<cplx, double>(p, p->stencil_d, p->m, 2, u, g, e, batch);
}
ls_status stencil_apply_A(ls_plan* p, const fcplx* r, fcplx* y, int batch) {
  return launch_stencil<fcplx, float>(p, p->f32.stencil, p->f32.m, 0, r, nullptr, y, batch);
}
ls_status stencil_apply_C(ls_plan* p, const fcplx* v, fcplx* y, int batch) {
  return launch_stencil<fcplx, float>(p, p->f32.stencil, p->f32.m, 1, v, nullptr, y, batch);
}
ls_status stencil_residual_C(ls_plan* p, const fcplx* g, const fcplx* u, fcplx* e, int batch) {
  return launch_stencil<fcplx, float>(p, p->f32.stencil, p->f32.m, 2, u, g, e, batch);
}
