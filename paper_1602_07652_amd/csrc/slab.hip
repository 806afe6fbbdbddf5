// Local slab problems and the polarized-traces sweeps.
//
// Section 3.1: layers Omega^l extended to Omega^l_ext; local problems
// C^l w^l = g^l.  Section 3.3: C^l is C on the layer (compatibility) with
// the perturbation multiplied by a cut-off xi^l (1 on the layer, a cubic
// spline to 0 over the extension) and the stencils of the boundary of
// Omega on the boundary of Omega^l_ext; an optional complex shift acts in
// the cut-off region.  Section 4.1: every local matrix is banded and
// factored once, independently (embarrassingly parallel).  Section 3.2,
// eq. (pde_GRF_real): traces enter a neighbour through the blocks
// C^l_{n,n+1}, C^l_{n+1,n}, C^l_{1,0}, C^l_{0,1}.  Alg. 1: downward sweep
// then upward sweep; Alg. 2: horizontal sweep, residual, vertical sweep.
//
// Layout of one extended slab (its own frame): long axis i in [0, n),
// short axis r in [0, q) for the line z0 + r.  Unknown (i, r) sits at
// i*q + r, so the matrix is block tridiagonal with q x q blocks along i
// (each block couples three lines of the short axis).  coef[i][r][9] holds
// C^l((i, r), (i+dX, r+dZ)) at slot (dZ+1)*3 + dX+1.
//
// Factorisation and solve: block cyclic reduction along the long axis
// (odd blocks eliminated level by level; level l holds the blocks
// i = k * 2^l), so one solve is ~2 log2(n) steps that are each parallel over
// the blocks of the level, instead of n sequential block steps.  Dense
// q x q blocks are stored column-major; inverses by Gauss-Jordan with
// partial pivoting.  Stored per level (k = level block index):
//   level 0   odd k : Dinv_k                          (L, U stay sparse in coef)
//   level l>0 odd k : Dinv_k, Dinv_k L_k, Dinv_k U_k
//             even k: Pm_k = L_k Dinv_{k-1}, Pp_k = U_k Dinv_{k+1}
//   last level (one block): Dinv.
// Solve (in place on b, layout [n][q]):
//   forward  level 0 : z_k = Dinv_k b_k (odd); b_k -= L_k z_{k-1} + U_k z_{k+1} (even)
//            level l : b_k -= Pm_k b_{k-1} + Pp_k b_{k+1} (even)
//   last             : x_0 = Dinv b_0
//   backward level l : x_k = Dinv_k b_k - (Dinv L)_k x_{k-1} - (Dinv U)_k x_{k+1} (odd)
//            level 0 : x_k = z_k - Dinv_k (L_k x_{k-1} + U_k x_{k+1}) (odd)
#include "ls_internal.h"

#include <algorithm>
#include <cmath>

namespace {

constexpr int kMaxQ = 96;
constexpr int kSolveThreads = 256;

__device__ __forceinline__ int axis_type(int i, int n) { return i == 0 ? 0 : (i == n - 1 ? 2 : 1); }

__device__ __forceinline__ double cutoff(int Z, int a, int b, int ext) {
  if (Z >= a - 1 && Z <= b + 1) return 1.0;
  const int dist = (Z < a) ? a - Z : Z - b;
  const double tau = (double)(dist - 1) / (double)(ext - 1);
  return 1.0 - 3.0 * tau * tau + 2.0 * tau * tau * tau;
}

__global__ void k_assemble(cplx* __restrict__ coef, const cplx* __restrict__ tables,
                           const double* __restrict__ m, int n, int q, int z0, int a, int b,
                           int ext, int orient, double omega2, double sigma) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y;
  if (r >= q) return;
  const int tX = axis_type(i, n);
  const int tZ = (r == 0) ? 0 : (r == q - 1 ? 2 : 1);
  const int t = tZ * 3 + tX;
  const cplx* al = tables + t * 9;
  const cplx* be = tables + 81 + t * 9;
  cplx* out = coef + ((size_t)i * q + r) * 9;
  for (int dZ = -1; dZ <= 1; ++dZ)
    for (int dX = -1; dX <= 1; ++dX) {
      const int s = (dZ + 1) * 3 + dX + 1;
      const int rr = r + dZ, ii = i + dX;
      cplx c = cmk(0.0, 0.0);
      if (rr >= 0 && rr < q && ii >= 0 && ii < n) {
        const int Z = z0 + rr;
        const double xi = cutoff(Z, a, b, ext);
        const double mv = (orient == 0) ? m[(size_t)Z * n + ii] : m[(size_t)ii * n + Z];
        const cplx D = cmk(xi * mv, sigma * (1.0 - xi));
        c = cadd(al[s], cmul(cscale(be[s], omega2), D));
      }
      out[s] = c;
    }
}

// Level-0 dense blocks (column-major): D_i, L_i (to i-1), U_i (to i+1).
__global__ void k_level0_blocks(const cplx* __restrict__ coef, int n, int q, cplx* __restrict__ D,
                                cplx* __restrict__ Lb, cplx* __restrict__ Ub) {
  const int i = blockIdx.x;
  const size_t qq = (size_t)q * q;
  for (int e = threadIdx.x; e < q * q; e += blockDim.x) {
    const int c = e / q, r = e % q;  // element (r, c) at c*q + r
    const int dZ = c - r;
    cplx d = cmk(0, 0), l = cmk(0, 0), u = cmk(0, 0);
    if (dZ >= -1 && dZ <= 1) {
      const cplx* cf = coef + ((size_t)i * q + r) * 9 + (dZ + 1) * 3;
      l = cf[0];
      d = cf[1];
      u = cf[2];
    }
    D[i * qq + e] = d;
    Lb[i * qq + e] = l;
    Ub[i * qq + e] = u;
  }
}

// Batched inverse by Gauss-Jordan with partial pivoting (|re|+|im|), the
// q x q matrix held in LDS.  One workgroup per matrix.
__global__ __launch_bounds__(256) void k_inverse(const cplx* const* __restrict__ src,
                                                 cplx* const* __restrict__ dst, int q,
                                                 int* __restrict__ status) {
  extern __shared__ cplx lds[];
  cplx* A = lds;                   // column-major q x q
  cplx* fcol = lds + q * q;        // saved column k
  cplx* prow = fcol + q;           // saved (scaled) row k
  int* piv = reinterpret_cast<int*>(prow + q);
  __shared__ int s_p;
  __shared__ int s_bad;
  const int tid = threadIdx.x, nt = blockDim.x;
  const cplx* S = src[blockIdx.x];
  cplx* Dm = dst[blockIdx.x];
  for (int e = tid; e < q * q; e += nt) A[e] = S[e];
  if (tid == 0) s_bad = 0;
  __syncthreads();
  for (int k = 0; k < q; ++k) {
    if (tid < 64) {
      double best = -1.0;
      int bi = k;
      for (int r = k + tid; r < q; r += 64) {
        const cplx v = A[k * q + r];
        const double mag = fabs(v.x) + fabs(v.y);
        if (mag > best) { best = mag; bi = r; }
      }
      for (int off = 32; off > 0; off >>= 1) {
        const double ob = __shfl_xor(best, off);
        const int oi = __shfl_xor(bi, off);
        if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
      }
      if (tid == 0) {
        s_p = bi;
        piv[k] = bi;
        if (!(best > 0.0) || !isfinite(best)) s_bad = 1;
      }
    }
    __syncthreads();
    const int p = s_p;
    if (p != k) {
      for (int c = tid; c < q; c += nt) {
        const cplx t = A[c * q + k];
        A[c * q + k] = A[c * q + p];
        A[c * q + p] = t;
      }
      __syncthreads();
    }
    const cplx pv = A[k * q + k];
    const double den = pv.x * pv.x + pv.y * pv.y;
    const cplx ip = cmk(pv.x / den, -pv.y / den);
    for (int r = tid; r < q; r += nt) fcol[r] = A[k * q + r];
    __syncthreads();
    for (int c = tid; c < q; c += nt) {
      const cplx v = (c == k) ? cmk(1.0, 0.0) : A[c * q + k];
      const cplx s = cmul(v, ip);
      prow[c] = s;
      A[c * q + k] = s;
    }
    __syncthreads();
    for (int e = tid; e < q * q; e += nt) {
      const int c = e / q, r = e % q;
      if (r == k) continue;
      const cplx base = (c == k) ? cmk(0.0, 0.0) : A[e];
      A[e] = csub(base, cmul(fcol[r], prow[c]));
    }
    __syncthreads();
  }
  for (int k = q - 1; k >= 0; --k) {
    const int p = piv[k];
    if (p != k) {
      for (int r = tid; r < q; r += nt) {
        const cplx t = A[k * q + r];
        A[k * q + r] = A[p * q + r];
        A[p * q + r] = t;
      }
    }
    __syncthreads();
  }
  for (int e = tid; e < q * q; e += nt) Dm[e] = A[e];
  if (tid == 0 && s_bad) atomicOr(status, 1);
}

// Batched C = Cin + alpha * A * B, all q x q column-major; Cin may be null
// (then C = alpha A B).  C may alias Cin.  32 x 32 output tile per
// workgroup, 2 x 2 per thread.
__global__ __launch_bounds__(256) void k_gemm(const cplx* const* __restrict__ Ap,
                                              const cplx* const* __restrict__ Bp,
                                              const cplx* const* __restrict__ Cinp,
                                              cplx* const* __restrict__ Cp, int q, cplx alpha) {
  __shared__ cplx As[16][33];
  __shared__ cplx Bs[16][33];
  const int b = blockIdx.y;
  const int tiles = (q + 31) / 32;
  const int tm = blockIdx.x % tiles, tn = blockIdx.x / tiles;
  const cplx* A = Ap[b];
  const cplx* B = Bp[b];
  const cplx* Cin = Cinp[b];
  cplx* C = Cp[b];
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
  cplx acc[2][2];
  for (int u = 0; u < 2; ++u)
    for (int v = 0; v < 2; ++v) acc[u][v] = cmk(0, 0);
  for (int k0 = 0; k0 < q; k0 += 16) {
    for (int e = threadIdx.x; e < 16 * 32; e += 256) {
      const int kk = e / 32, rr = e % 32;
      const int gr = tm * 32 + rr, gk = k0 + kk;
      As[kk][rr] = (gr < q && gk < q) ? A[(size_t)gk * q + gr] : cmk(0, 0);  // A(gr, gk)
      const int cc = e % 32, kb = e / 32;
      const int gc = tn * 32 + cc, gkb = k0 + kb;
      Bs[kb][cc] = (gc < q && gkb < q) ? B[(size_t)gc * q + gkb] : cmk(0, 0);  // B(gkb, gc)
    }
    __syncthreads();
#pragma unroll 4
    for (int kk = 0; kk < 16; ++kk) {
      const cplx a0 = As[kk][ty * 2], a1 = As[kk][ty * 2 + 1];
      const cplx b0 = Bs[kk][tx * 2], b1 = Bs[kk][tx * 2 + 1];
      acc[0][0] = cfma(a0, b0, acc[0][0]);
      acc[0][1] = cfma(a0, b1, acc[0][1]);
      acc[1][0] = cfma(a1, b0, acc[1][0]);
      acc[1][1] = cfma(a1, b1, acc[1][1]);
    }
    __syncthreads();
  }
  for (int u = 0; u < 2; ++u)
    for (int v = 0; v < 2; ++v) {
      const int gr = tm * 32 + ty * 2 + u, gc = tn * 32 + tx * 2 + v;
      if (gr < q && gc < q) {
        const size_t idx = (size_t)gc * q + gr;
        cplx val = cmul(alpha, acc[u][v]);
        if (Cin) val = cadd(Cin[idx], val);
        C[idx] = val;
      }
    }
}

// ------------------------------------------------------------ solve kernels
struct GemvLane {
  int r, c0, c1, cs, CS;
};

__device__ __forceinline__ GemvLane gemv_lane(int q, int tid) {
  GemvLane g;
  const int RH = (q + 63) / 64;
  g.CS = 4 / RH;
  const int w = tid >> 6, lane = tid & 63;
  const int rh = w % RH;
  g.cs = w / RH;
  g.r = rh * 64 + lane;
  const int chunk = (q + g.CS - 1) / g.CS;
  g.c0 = g.cs * chunk;
  g.c1 = min(q, g.c0 + chunk);
  return g;
}

// acc += M(r, c0:c1) * x(c0:c1), M column-major q x q.
__device__ __forceinline__ cplx gemv_part(const cplx* __restrict__ M, const cplx* x, int q,
                                          const GemvLane& g, cplx acc) {
  if (g.r < q) {
    const cplx* col = M + g.r;
#pragma unroll 8
    for (int c = g.c0; c < g.c1; ++c) acc = cfma(col[(size_t)c * q], x[c], acc);
  }
  return acc;
}

// Sum the column splits; returns the result for row tid (valid if tid < q).
__device__ __forceinline__ cplx gemv_reduce(cplx acc, const GemvLane& g, cplx* part, int q) {
  if (g.r < q) part[g.cs * 128 + g.r] = acc;
  __syncthreads();
  cplx y = cmk(0, 0);
  if (threadIdx.x < q)
    for (int s = 0; s < g.CS; ++s) y = cadd(y, part[s * 128 + threadIdx.x]);
  return y;
}

__global__ __launch_bounds__(kSolveThreads) void k_fwd0_odd(cplx* __restrict__ x,
                                                            const cplx* __restrict__ dinv, int q) {
  __shared__ cplx xs[kMaxQ];
  __shared__ cplx part[4 * 128];
  const int k = 2 * blockIdx.x + 1;
  const size_t qq = (size_t)q * q;
  if (threadIdx.x < q) xs[threadIdx.x] = x[(size_t)k * q + threadIdx.x];
  __syncthreads();
  const GemvLane g = gemv_lane(q, threadIdx.x);
  cplx acc = gemv_part(dinv + blockIdx.x * qq, xs, q, g, cmk(0, 0));
  const cplx y = gemv_reduce(acc, g, part, q);
  if (threadIdx.x < q) x[(size_t)k * q + threadIdx.x] = y;
}

__global__ void k_fwd0_even(cplx* __restrict__ x, const cplx* __restrict__ coef, int n, int q) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  const int k = 2 * blockIdx.y;
  if (r >= q) return;
  const cplx* cf = coef + ((size_t)k * q + r) * 9;
  cplx acc = x[(size_t)k * q + r];
  for (int dZ = -1; dZ <= 1; ++dZ) {
    const int rr = r + dZ;
    if (rr < 0 || rr >= q) continue;
    if (k >= 1) acc = csub(acc, cmul(cf[(dZ + 1) * 3 + 0], x[(size_t)(k - 1) * q + rr]));
    if (k + 1 < n) acc = csub(acc, cmul(cf[(dZ + 1) * 3 + 2], x[(size_t)(k + 1) * q + rr]));
  }
  x[(size_t)k * q + r] = acc;
}

__global__ __launch_bounds__(kSolveThreads) void k_fwd(cplx* __restrict__ x,
                                                       const cplx* __restrict__ pm,
                                                       const cplx* __restrict__ pp, int q, int nl,
                                                       int shift) {
  __shared__ cplx xm[kMaxQ], xp[kMaxQ];
  __shared__ cplx part[4 * 128];
  const int k = 2 * blockIdx.x;
  const size_t qq = (size_t)q * q;
  const bool hm = k >= 1, hp = k + 1 < nl;
  if (threadIdx.x < q) {
    xm[threadIdx.x] = hm ? x[((size_t)(k - 1) << shift) * q + threadIdx.x] : cmk(0, 0);
    xp[threadIdx.x] = hp ? x[((size_t)(k + 1) << shift) * q + threadIdx.x] : cmk(0, 0);
  }
  __syncthreads();
  const GemvLane g = gemv_lane(q, threadIdx.x);
  cplx acc = cmk(0, 0);
  if (hm) acc = gemv_part(pm + blockIdx.x * qq, xm, q, g, acc);
  if (hp) acc = gemv_part(pp + blockIdx.x * qq, xp, q, g, acc);
  const cplx y = gemv_reduce(acc, g, part, q);
  if (threadIdx.x < q) {
    const size_t o = ((size_t)k << shift) * q + threadIdx.x;
    x[o] = csub(x[o], y);
  }
}

__global__ __launch_bounds__(kSolveThreads) void k_last(cplx* __restrict__ x,
                                                        const cplx* __restrict__ dinv, int q) {
  __shared__ cplx xs[kMaxQ];
  __shared__ cplx part[4 * 128];
  if (threadIdx.x < q) xs[threadIdx.x] = x[threadIdx.x];
  __syncthreads();
  const GemvLane g = gemv_lane(q, threadIdx.x);
  const cplx y = gemv_reduce(gemv_part(dinv, xs, q, g, cmk(0, 0)), g, part, q);
  if (threadIdx.x < q) x[threadIdx.x] = y;
}

__global__ __launch_bounds__(kSolveThreads) void k_bwd(cplx* __restrict__ x,
                                                       const cplx* __restrict__ dinv,
                                                       const cplx* __restrict__ dinvl,
                                                       const cplx* __restrict__ dinvu, int q,
                                                       int nl, int shift) {
  __shared__ cplx xb[kMaxQ], xm[kMaxQ], xp[kMaxQ];
  __shared__ cplx part[4 * 128];
  const int k = 2 * blockIdx.x + 1;
  const size_t qq = (size_t)q * q;
  const bool hp = k + 1 < nl;
  if (threadIdx.x < q) {
    xb[threadIdx.x] = x[((size_t)k << shift) * q + threadIdx.x];
    const cplx a = x[((size_t)(k - 1) << shift) * q + threadIdx.x];
    xm[threadIdx.x] = cmk(-a.x, -a.y);
    if (hp) {
      const cplx c = x[((size_t)(k + 1) << shift) * q + threadIdx.x];
      xp[threadIdx.x] = cmk(-c.x, -c.y);
    }
  }
  __syncthreads();
  const GemvLane g = gemv_lane(q, threadIdx.x);
  cplx acc = gemv_part(dinv + blockIdx.x * qq, xb, q, g, cmk(0, 0));
  acc = gemv_part(dinvl + blockIdx.x * qq, xm, q, g, acc);
  if (hp) acc = gemv_part(dinvu + blockIdx.x * qq, xp, q, g, acc);
  const cplx y = gemv_reduce(acc, g, part, q);
  if (threadIdx.x < q) x[((size_t)k << shift) * q + threadIdx.x] = y;
}

__global__ __launch_bounds__(kSolveThreads) void k_bwd0(cplx* __restrict__ x,
                                                        const cplx* __restrict__ dinv,
                                                        const cplx* __restrict__ coef, int n,
                                                        int q) {
  __shared__ cplx t[kMaxQ];
  __shared__ cplx part[4 * 128];
  const int k = 2 * blockIdx.x + 1;
  const size_t qq = (size_t)q * q;
  const int r = threadIdx.x;
  if (r < q) {
    const cplx* cf = coef + ((size_t)k * q + r) * 9;
    cplx acc = cmk(0, 0);
    for (int dZ = -1; dZ <= 1; ++dZ) {
      const int rr = r + dZ;
      if (rr < 0 || rr >= q) continue;
      acc = cfma(cf[(dZ + 1) * 3 + 0], x[(size_t)(k - 1) * q + rr], acc);
      if (k + 1 < n) acc = cfma(cf[(dZ + 1) * 3 + 2], x[(size_t)(k + 1) * q + rr], acc);
    }
    t[r] = acc;
  }
  __syncthreads();
  const GemvLane g = gemv_lane(q, threadIdx.x);
  const cplx y = gemv_reduce(gemv_part(dinv + blockIdx.x * qq, t, q, g, cmk(0, 0)), g, part, q);
  if (threadIdx.x < q) {
    const size_t o = (size_t)k * q + threadIdx.x;
    x[o] = csub(x[o], y);
  }
}

// ------------------------------------------------------- sweep helpers
// dst[i][r] = g(i, z0 + r) on the layer lines [a, b], 0 elsewhere.
__global__ void k_gather(const cplx* __restrict__ g, cplx* __restrict__ dst, int n, int q, int z0,
                         int a, int b, int orient) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * q) return;
  int i, r;
  if (orient == 0) { r = t / n; i = t % n; } else { i = t / q; r = t % q; }
  const int Z = z0 + r;
  cplx v = cmk(0, 0);
  if (Z >= a && Z <= b) v = (orient == 0) ? g[(size_t)Z * n + i] : g[(size_t)i * n + Z];
  dst[(size_t)i * q + r] = v;
}

// out(i, Z) (+)= src[i][Z - z0] for Z in [a, b].
__global__ void k_scatter(const cplx* __restrict__ src, cplx* __restrict__ out, int n, int q,
                          int z0, int a, int b, int orient, int accumulate) {
  const int rows = b - a + 1;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * rows) return;
  int i, Z;
  if (orient == 0) { Z = a + t / n; i = t % n; } else { i = t / rows; Z = a + t % rows; }
  const cplx v = src[(size_t)i * q + (Z - z0)];
  const size_t o = (orient == 0) ? (size_t)Z * n + i : (size_t)i * n + Z;
  out[o] = accumulate ? cadd(out[o], v) : v;
}

// GRF source: rhs[i][rt] += sgn * sum_dX coef[i][rt][(dZ+1)*3 + dX+1] *
// (s1[(i+dX)*q1 + r1] + s2[(i+dX)*q2 + r2]).
__global__ void k_inject(cplx* __restrict__ rhs, const cplx* __restrict__ coef, int n, int q,
                         int rt, int dZ, double sgn, const cplx* __restrict__ s1, int q1, int r1,
                         const cplx* __restrict__ s2, int q2, int r2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const cplx* cf = coef + ((size_t)i * q + rt) * 9 + (dZ + 1) * 3;
  cplx acc = cmk(0, 0);
  for (int dX = -1; dX <= 1; ++dX) {
    const int ii = i + dX;
    if (ii < 0 || ii >= n) continue;
    cplx s = s1[(size_t)ii * q1 + r1];
    if (s2) s = cadd(s, s2[(size_t)ii * q2 + r2]);
    acc = cfma(cf[dX + 1], s, acc);
  }
  cplx* o = rhs + (size_t)i * q + rt;
  *o = cadd(*o, cscale(acc, sgn));
}

template <typename K>
hipError_t set_lds(K kernel, size_t bytes) {
  if (bytes <= 65536) return hipSuccess;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

struct PtrBatch {
  std::vector<const cplx*> a, b, cin;
  std::vector<cplx*> c;
};

// Device copies of pointer arrays (grown on demand).
struct DevPtrs {
  void* buf = nullptr;
  size_t cap = 0;
  ~DevPtrs() { if (buf) (void)hipFree(buf); }
};

ls_status run_gemm(ls_plan* p, DevPtrs& dp, const PtrBatch& pb, int q, cplx alpha) {
  const size_t cnt = pb.c.size();
  if (cnt == 0) return LS_OK;
  const size_t bytes = 4 * cnt * sizeof(void*);
  if (dp.cap < bytes) {
    if (dp.buf) LS_HIP(hipFree(dp.buf));
    LS_HIP(hipMalloc(&dp.buf, bytes));
    dp.cap = bytes;
  }
  std::vector<const void*> h(4 * cnt);
  for (size_t i = 0; i < cnt; ++i) {
    h[i] = pb.a[i];
    h[cnt + i] = pb.b[i];
    h[2 * cnt + i] = pb.cin[i];
    h[3 * cnt + i] = pb.c[i];
  }
  LS_HIP(hipMemcpyAsync(dp.buf, h.data(), bytes, hipMemcpyHostToDevice, p->stream));
  void** d = reinterpret_cast<void**>(dp.buf);
  const int tiles = (q + 31) / 32;
  for (size_t s = 0; s < cnt; s += 65535) {
    const int nb = (int)std::min<size_t>(65535, cnt - s);
    k_gemm<<<dim3(tiles * tiles, nb), 256, 0, p->stream>>>(
        reinterpret_cast<const cplx* const*>(d) + s, reinterpret_cast<const cplx* const*>(d + cnt) + s,
        reinterpret_cast<const cplx* const*>(d + 2 * cnt) + s,
        reinterpret_cast<cplx* const*>(d + 3 * cnt) + s, q, alpha);
    LS_HIP(hipGetLastError());
  }
  // the pointer array is reused by the next call: wait for this one
  LS_HIP(hipStreamSynchronize(p->stream));
  return LS_OK;
}

ls_status run_inverse(ls_plan* p, DevPtrs& dp, const std::vector<const cplx*>& src,
                      const std::vector<cplx*>& dst, int q, int* status) {
  const size_t cnt = src.size();
  if (cnt == 0) return LS_OK;
  const size_t bytes = 2 * cnt * sizeof(void*);
  if (dp.cap < bytes) {
    if (dp.buf) LS_HIP(hipFree(dp.buf));
    LS_HIP(hipMalloc(&dp.buf, bytes));
    dp.cap = bytes;
  }
  std::vector<const void*> h(2 * cnt);
  for (size_t i = 0; i < cnt; ++i) {
    h[i] = src[i];
    h[cnt + i] = dst[i];
  }
  LS_HIP(hipMemcpyAsync(dp.buf, h.data(), bytes, hipMemcpyHostToDevice, p->stream));
  const size_t lds = (size_t)q * q * sizeof(cplx) + 2 * q * sizeof(cplx) + q * sizeof(int) + 64;
  LS_HIP(set_lds(k_inverse, lds));
  void** d = reinterpret_cast<void**>(dp.buf);
  for (size_t s = 0; s < cnt; s += 65535) {
    const int nb = (int)std::min<size_t>(65535, cnt - s);
    k_inverse<<<nb, 256, lds, p->stream>>>(reinterpret_cast<const cplx* const*>(d) + s,
                                           reinterpret_cast<cplx* const*>(d + cnt) + s, q, status);
    LS_HIP(hipGetLastError());
  }
  LS_HIP(hipStreamSynchronize(p->stream));
  return LS_OK;
}

// Plan the factor storage of one slab.
size_t plan_levels(Slab& s, int n) {
  const size_t qq = (size_t)s.q * s.q;
  size_t off = 0;
  int nl = n;
  s.levels.clear();
  for (int l = 0;; ++l) {
    SlabLevel L{};
    L.nl = nl;
    L.off_dinvl = L.off_dinvu = L.off_pm = L.off_pp = (size_t)-1;
    if (nl == 1) {
      L.off_dinv = off;
      off += qq;
      s.levels.push_back(L);
      break;
    }
    const int no = nl / 2, ne = (nl + 1) / 2;
    L.off_dinv = off;
    off += no * qq;
    if (l > 0) {
      L.off_dinvl = off;
      off += no * qq;
      L.off_dinvu = off;
      off += no * qq;
      L.off_pm = off;
      off += ne * qq;
      L.off_pp = off;
      off += ne * qq;
    }
    s.levels.push_back(L);
    nl = ne;
  }
  return off;
}

// Factor one slab by block cyclic reduction.  work: 6 * n * q^2 + (n/2+1)*2*q^2
// complex of scratch.
ls_status factor_slab(ls_plan* p, Slab& s, cplx* work, int* status) {
  const int n = p->n, q = s.q;
  const size_t qq = (size_t)q * q;
  cplx* D = work;
  cplx* Lb = D + (size_t)n * qq;
  cplx* Ub = Lb + (size_t)n * qq;
  const size_t half = (size_t)(n / 2 + 1) * qq;
  cplx* Dn = Ub + (size_t)n * qq;
  cplx* Ln = Dn + half;
  cplx* Un = Ln + half;
  cplx* Pm0 = Un + half;   // level-0 temporaries
  cplx* Pp0 = Pm0 + half;
  k_level0_blocks<<<n, 256, 0, p->stream>>>(s.coef, n, q, D, Lb, Ub);
  LS_HIP(hipGetLastError());
  DevPtrs dp;
  const cplx one = cmk(1, 0), mone = cmk(-1, 0);
  for (size_t l = 0; l < s.levels.size(); ++l) {
    const SlabLevel& L = s.levels[l];
    const int nl = L.nl;
    cplx* fac = s.fac;
    if (nl == 1) {
      std::vector<const cplx*> src{D};
      std::vector<cplx*> dst{fac + L.off_dinv};
      LS_TRY(run_inverse(p, dp, src, dst, q, status));
      break;
    }
    const int no = nl / 2, ne = (nl + 1) / 2;
    auto blk = [&](cplx* base, int k) { return base + (size_t)k * qq; };
    {
      std::vector<const cplx*> src;
      std::vector<cplx*> dst;
      for (int j = 0; j < no; ++j) {
        src.push_back(blk(D, 2 * j + 1));
        dst.push_back(fac + L.off_dinv + (size_t)j * qq);
      }
      LS_TRY(run_inverse(p, dp, src, dst, q, status));
    }
    auto dinv = [&](int k) { return fac + L.off_dinv + (size_t)(k / 2) * qq; };
    if (l > 0) {
      PtrBatch pb;
      for (int j = 0; j < no; ++j) {
        const int k = 2 * j + 1;
        pb.a.push_back(dinv(k)); pb.b.push_back(blk(Lb, k)); pb.cin.push_back(nullptr);
        pb.c.push_back(fac + L.off_dinvl + (size_t)j * qq);
        pb.a.push_back(dinv(k)); pb.b.push_back(blk(Ub, k)); pb.cin.push_back(nullptr);
        pb.c.push_back(fac + L.off_dinvu + (size_t)j * qq);
      }
      LS_TRY(run_gemm(p, dp, pb, q, one));
    }
    cplx* PM = (l > 0) ? fac + L.off_pm : Pm0;
    cplx* PP = (l > 0) ? fac + L.off_pp : Pp0;
    LS_HIP(hipMemsetAsync(PM, 0, ne * qq * sizeof(cplx), p->stream));
    LS_HIP(hipMemsetAsync(PP, 0, ne * qq * sizeof(cplx), p->stream));
    {
      PtrBatch pb;
      for (int j = 0; j < ne; ++j) {
        const int k = 2 * j;
        if (k >= 1) {
          pb.a.push_back(blk(Lb, k)); pb.b.push_back(dinv(k - 1)); pb.cin.push_back(nullptr);
          pb.c.push_back(PM + (size_t)j * qq);
        }
        if (k + 1 < nl) {
          pb.a.push_back(blk(Ub, k)); pb.b.push_back(dinv(k + 1)); pb.cin.push_back(nullptr);
          pb.c.push_back(PP + (size_t)j * qq);
        }
      }
      LS_TRY(run_gemm(p, dp, pb, q, one));
    }
    LS_HIP(hipMemsetAsync(Ln, 0, ne * qq * sizeof(cplx), p->stream));
    LS_HIP(hipMemsetAsync(Un, 0, ne * qq * sizeof(cplx), p->stream));
    {
      // Dn = D_k - Pm U_{k-1}; Ln = -Pm L_{k-1}; Un = -Pp U_{k+1}
      PtrBatch pb;
      for (int j = 0; j < ne; ++j) {
        const int k = 2 * j;
        if (k >= 1) {
          pb.a.push_back(PM + (size_t)j * qq); pb.b.push_back(blk(Ub, k - 1));
          pb.cin.push_back(blk(D, k)); pb.c.push_back(Dn + (size_t)j * qq);
          pb.a.push_back(PM + (size_t)j * qq); pb.b.push_back(blk(Lb, k - 1));
          pb.cin.push_back(nullptr); pb.c.push_back(Ln + (size_t)j * qq);
        }
        if (k + 1 < nl) {
          pb.a.push_back(PP + (size_t)j * qq); pb.b.push_back(blk(Ub, k + 1));
          pb.cin.push_back(nullptr); pb.c.push_back(Un + (size_t)j * qq);
        }
        if (k < 1) {
          // no left neighbour: Dn starts from D_k
          pb.a.push_back(PP + (size_t)j * qq); pb.b.push_back(blk(Lb, k + 1));
          pb.cin.push_back(blk(D, k)); pb.c.push_back(Dn + (size_t)j * qq);
        }
      }
      LS_TRY(run_gemm(p, dp, pb, q, mone));
    }
    {
      // Dn -= Pp L_{k+1} for blocks that had a left neighbour
      PtrBatch pb;
      for (int j = 0; j < ne; ++j) {
        const int k = 2 * j;
        if (k >= 1 && k + 1 < nl) {
          pb.a.push_back(PP + (size_t)j * qq); pb.b.push_back(blk(Lb, k + 1));
          pb.cin.push_back(Dn + (size_t)j * qq); pb.c.push_back(Dn + (size_t)j * qq);
        }
      }
      LS_TRY(run_gemm(p, dp, pb, q, mone));
    }
    // next level
    LS_HIP(hipMemcpyAsync(D, Dn, ne * qq * sizeof(cplx), hipMemcpyDeviceToDevice, p->stream));
    LS_HIP(hipMemcpyAsync(Lb, Ln, ne * qq * sizeof(cplx), hipMemcpyDeviceToDevice, p->stream));
    LS_HIP(hipMemcpyAsync(Ub, Un, ne * qq * sizeof(cplx), hipMemcpyDeviceToDevice, p->stream));
  }
  LS_HIP(hipStreamSynchronize(p->stream));
  return LS_OK;
}

}  // namespace

// Layers (Section 3.1): t = n / L lines each, the first n mod L layers one
// more; extension ext lines each side, clipped to the grid.
ls_status slabs_build(ls_plan* p) {
  const int n = p->n, L = p->L, ext = p->opt.ext;
  const int t = n / L, rem = n % L;
  int qmax = 0;
  for (int o = 0; o < 2; ++o) {
    p->slabs[o].clear();
    int a = 0;
    for (int l = 0; l < L; ++l) {
      Slab s{};
      s.orient = o;
      s.idx = l;
      s.a = a;
      s.b = a + (l < rem ? t + 1 : t) - 1;
      s.z0 = std::max(0, s.a - ext);
      s.z1 = std::min(n - 1, s.b + ext);
      s.q = s.z1 - s.z0 + 1;
      a = s.b + 1;
      qmax = std::max(qmax, s.q);
      p->slabs[o].push_back(s);
    }
  }
  if (qmax > kMaxQ) {
    ls_set_error("extended layer thickness q = " + std::to_string(qmax) + " exceeds " +
                 std::to_string(kMaxQ) + "; use more slabs or a smaller extension");
    return LS_EUNSUPPORTED;
  }
  // scratch for the factorisation (largest q)
  const size_t qq = (size_t)qmax * qmax;
  const size_t work_elems = 3 * (size_t)n * qq + 5 * (size_t)(n / 2 + 1) * qq;
  cplx* work = nullptr;
  int* status = nullptr;
  LS_HIP(hipMalloc(&work, work_elems * sizeof(cplx)));
  LS_HIP(hipMalloc(&status, sizeof(int)));
  LS_HIP(hipMemsetAsync(status, 0, sizeof(int), p->stream));
  const double w2 = p->omega * p->omega;
  const double sigma = p->opt.shift_c / p->omega;
  ls_status st = LS_OK;
  for (int o = 0; o < 2 && st == LS_OK; ++o) {
    for (Slab& s : p->slabs[o]) {
      const size_t cbytes = (size_t)n * s.q * 9 * sizeof(cplx);
      if ((st = plan_alloc(p, (void**)&s.coef, cbytes)) != LS_OK) break;
      if ((st = plan_alloc(p, (void**)&s.g, (size_t)n * s.q * sizeof(cplx))) != LS_OK) break;
      if ((st = plan_alloc(p, (void**)&s.w, (size_t)n * s.q * sizeof(cplx))) != LS_OK) break;
      s.fac_elems = plan_levels(s, n);
      if ((st = plan_alloc(p, (void**)&s.fac, s.fac_elems * sizeof(cplx))) != LS_OK) break;
      const cplx* tables = p->stencil_d + (o == 0 ? 0 : 162);
      k_assemble<<<dim3((s.q + 63) / 64, n), 64, 0, p->stream>>>(
          s.coef, tables, p->m, n, s.q, s.z0, s.a, s.b, std::max(ext, 2), o, w2, sigma);
      if (hipGetLastError() != hipSuccess) { ls_set_error("assembly launch failed"); st = LS_EDEVICE; break; }
      if ((st = factor_slab(p, s, work, status)) != LS_OK) break;
    }
  }
  int bad = 0;
  if (st == LS_OK) {
    if (hipMemcpy(&bad, status, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess) st = LS_EDEVICE;
  }
  (void)hipFree(work);
  (void)hipFree(status);
  if (st != LS_OK) return st;
  if (bad) {
    ls_set_error("slab factorisation: zero or non-finite pivot");
    return LS_ESINGULAR;
  }
  LS_TRY(plan_alloc(p, (void**)&p->slab_work, (size_t)n * qmax * sizeof(cplx)));
  LS_TRY(plan_alloc(p, (void**)&p->slab_work2, (size_t)n * qmax * sizeof(cplx)));
  return LS_OK;
}

ls_status slab_solve_frame(ls_plan* p, Slab& s, cplx* x) {
  const int n = p->n, q = s.q;
  const size_t qq = (size_t)q * q;
  const cplx* fac = s.fac;
  const int nlev = (int)s.levels.size();
  if (nlev == 1) {
    k_last<<<1, kSolveThreads, 0, p->stream>>>(x, fac + s.levels[0].off_dinv, q);
    LS_HIP(hipGetLastError());
    return LS_OK;
  }
  (void)qq;
  // forward
  const SlabLevel& L0 = s.levels[0];
  k_fwd0_odd<<<L0.nl / 2, kSolveThreads, 0, p->stream>>>(x, fac + L0.off_dinv, q);
  k_fwd0_even<<<dim3((q + 127) / 128, (L0.nl + 1) / 2), 128, 0, p->stream>>>(x, s.coef, n, q);
  for (int l = 1; l < nlev - 1; ++l) {
    const SlabLevel& L = s.levels[l];
    k_fwd<<<(L.nl + 1) / 2, kSolveThreads, 0, p->stream>>>(x, fac + L.off_pm, fac + L.off_pp, q,
                                                         L.nl, l);
  }
  k_last<<<1, kSolveThreads, 0, p->stream>>>(x, fac + s.levels[nlev - 1].off_dinv, q);
  for (int l = nlev - 2; l >= 1; --l) {
    const SlabLevel& L = s.levels[l];
    k_bwd<<<L.nl / 2, kSolveThreads, 0, p->stream>>>(x, fac + L.off_dinv, fac + L.off_dinvl,
                                                   fac + L.off_dinvu, q, L.nl, l);
  }
  k_bwd0<<<L0.nl / 2, kSolveThreads, 0, p->stream>>>(x, fac + L0.off_dinv, s.coef, n, q);
  LS_HIP(hipGetLastError());
  return LS_OK;
}

static ls_status gather(ls_plan* p, const Slab& s, const cplx* g, cplx* dst) {
  const int n = p->n, tot = n * s.q;
  k_gather<<<(tot + 255) / 256, 256, 0, p->stream>>>(g, dst, n, s.q, s.z0, s.a, s.b, s.orient);
  LS_HIP(hipGetLastError());
  return LS_OK;
}

static ls_status scatter(ls_plan* p, const Slab& s, const cplx* src, cplx* out, bool acc) {
  const int n = p->n, tot = n * (s.b - s.a + 1);
  k_scatter<<<(tot + 255) / 256, 256, 0, p->stream>>>(src, out, n, s.q, s.z0, s.a, s.b,
                                                      s.orient, acc ? 1 : 0);
  LS_HIP(hipGetLastError());
  return LS_OK;
}

static ls_status inject(ls_plan* p, const Slab& s, cplx* rhs, int line, int dZ, double sgn,
                        const cplx* s1, const Slab& o1, int line1, const cplx* s2,
                        const Slab* o2, int line2) {
  const int n = p->n;
  k_inject<<<(n + 255) / 256, 256, 0, p->stream>>>(
      rhs, s.coef, n, s.q, line - s.z0, dZ, sgn, s1, o1.q, line1 - o1.z0, s2,
      o2 ? o2->q : 0, o2 ? line2 - o2->z0 : 0);
  LS_HIP(hipGetLastError());
  return LS_OK;
}

// Alg. 1 (Gauss-Seidel polarized traces) on layers of one orientation.
// v receives the concatenated layer solutions (or has them added).
ls_status sweep_apply(ls_plan* p, int orient, const cplx* g, cplx* v, bool accumulate) {
  std::vector<Slab>& S = p->slabs[orient];
  const int L = (int)S.size();
  const int n = p->n;
  // downward sweep: l = L-1 .. 0
  for (int l = L - 1; l >= 0; --l) {
    Slab& s = S[l];
    LS_TRY(gather(p, s, g, s.g));
    if (l != L - 1) {
      const Slab& up = S[l + 1];
      // g^l += -delta_b C^l_{b,b+1} w^{l+1}(b+1) + delta_{b+1} C^l_{b+1,b} w^{l+1}(b)
      LS_TRY(inject(p, s, s.g, s.b, +1, -1.0, up.w, up, s.b + 1, nullptr, nullptr, 0));
      LS_TRY(inject(p, s, s.g, s.b + 1, -1, +1.0, up.w, up, s.b, nullptr, nullptr, 0));
    }
    LS_HIP(hipMemcpyAsync(s.w, s.g, (size_t)n * s.q * sizeof(cplx), hipMemcpyDeviceToDevice,
                          p->stream));
    LS_TRY(slab_solve_frame(p, s, s.w));
  }
  // upward sweep: l = 0 .. L-1
  cplx* vprev = p->slab_work;
  cplx* vcur = p->slab_work2;
  for (int l = 0; l < L; ++l) {
    Slab& s = S[l];
    if (l == 0) {
      // g^0 is unchanged: v^0 = w^0
      LS_HIP(hipMemcpyAsync(vcur, s.w, (size_t)n * s.q * sizeof(cplx), hipMemcpyDeviceToDevice,
                            p->stream));
    } else {
      const Slab& dn = S[l - 1];
      // g^l += -delta_a C^l_{a,a-1} v0 + delta_{a-1} C^l_{a-1,a} v1 with
      // v0 = v^{l-1}(a-1), v1 = v^{l-1}(a) + w^l(a)
      LS_TRY(inject(p, s, s.g, s.a, -1, -1.0, vprev, dn, s.a - 1, nullptr, nullptr, 0));
      LS_TRY(inject(p, s, s.g, s.a - 1, +1, +1.0, vprev, dn, s.a, s.w, &s, s.a));
      LS_HIP(hipMemcpyAsync(vcur, s.g, (size_t)n * s.q * sizeof(cplx), hipMemcpyDeviceToDevice,
                            p->stream));
      LS_TRY(slab_solve_frame(p, s, vcur));
    }
    LS_TRY(scatter(p, s, vcur, v, accumulate));
    std::swap(vprev, vcur);
  }
  return LS_OK;
}

// Alg. 2: u1 = Prec_H(g); e = g - C u1; u2 = Prec_V(e); v = u1 + u2.
ls_status bidirectional_apply(ls_plan* p, const cplx* g, cplx* v) {
  cplx* e = p->vtmp;
  LS_TRY(sweep_apply(p, 0, g, v, false));
  LS_TRY(stencil_residual_C(p, g, v, e));
  LS_TRY(sweep_apply(p, 1, e, v, true));
  return LS_OK;
}
