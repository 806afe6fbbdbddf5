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
#include <cstring>
#include <cmath>
#include <mutex>

namespace {

constexpr int kMaxQ = 96;

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

// consecutive logical workgroups (the tiles of one block) on one XCD
__device__ __forceinline__ int bstep_remap(int id, int total) {
  const int per = total / 8;
  if (per == 0 || id >= per * 8) return id;
  return (id % 8) * per + id / 8;
}

// ------------------------------------------------------------ solve kernels
// Single right-hand side.  The solve reads the right-hand side g, keeps the
// eliminated right-hand sides of the even block rows in a scratch t, and
// writes the solution to y (g, t, y: [n][q] slab frames), so no launch reads
// a row it also writes: a block's output rows can then be split over
// several workgroups.  Every level step is y_k = sum_t M_t x_t over up to
// three q x q column-major matrices of block k.
//
// Workgroup (block, row tile): rows [r0, r0 + R) of the block, R = q / RS.
// Thread (rl, grp) = (tid % R, tid / R) takes the virtual columns v = grp,
// grp + G, ... (G = 256 / R) of the T*q columns and loads all its factor
// elements (at most RCols::N) into registers before anything else, so a
// level costs about one memory round trip however deep it is; the inputs
// x_t are staged in LDS meanwhile and the G partial sums added in LDS.
enum { R_ODD0 = 0, R_FWD = 1, R_LAST = 2, R_BWD = 3, R_BWD0 = 4, R_BWD0S = 5, R_BWD0R = 6, R_ODDL = 7 };
// factor columns a thread preloads: one, two or three matrices per step
template <int MODE>
struct RCols {
  static constexpr int T = MODE == R_BWD ? 3 : (MODE == R_FWD ? 2 : 1);
  static constexpr int N = 7 * T;
};

// Row tiles per block for `rows` rows of factor matrices with q columns:
// the fewest with at most ncol columns per thread for a step with t
// factor matrices (rows = q: whole blocks).
inline int row_splits(int rows, int q, int t, int ncol) {
  for (int rs = 1; rs <= rows; ++rs) {
    const int R = (rows + rs - 1) / rs, G = 256 / R;
    if (G >= 1 && (t * q + G - 1) / G <= ncol) return rs;
  }
  return rows;
}
inline int row_splits(int q, int t, int ncol) { return row_splits(q, q, t, ncol); }

// Modes (k: block row at this level, rows of level l are global rows k<<l):
//   R_ODD0  level 0, k odd:  y_k = Dinv_k g_k
//   R_FWD   level l, k even: t_k -= Pm_k t_{k-1} + Pp_k t_{k+1}
//   R_LAST  top level:       y_0 = Dinv t_0
//   R_BWD   level l, k odd:  y_k = Dinv_k t_k - (Dinv L)_k y_{k-1} - (Dinv U)_k y_{k+1}
//   R_BWD0  level 0, k odd:  y_k -= Dinv_k t_k, t_k = L_k y_{k-1} + U_k y_{k+1} (k_odd0_lu)
//   R_BWD0S as R_BWD0 for the rows S.sel[slab] only (at most 4, -1 = none; one
//           row tile per block): the other rows of the odd blocks keep the
//           level-0 forward values
//   R_BWD0R as R_BWD0 for the rows [S.lo[slab], S.hi[slab]) only (RS tiles)
//   R_ODDL  level l, k odd:  y_k = Dinv_k t_k
// Slabs of one launch: the one-right-hand-side steps run the same level
// step (same q and level structure: the factor blocks of a level at the
// same offsets) for up to kSet slabs at once, blockIdx.y (k_rstep, k_top)
// or blockIdx.z (k_even0, k_odd0_lu) picking the slab; a single solve is a
// set of one.
constexpr int kSet = 16;
template <typename C>
struct SlabSet {
  const C* g[kSet];    // right-hand sides [n][q]
  C* t[kSet];          // elimination scratch [n][q]
  C* y[kSet];          // solutions [n][q]
  const C* fac[kSet];  // factors (level offsets shared by the set)
  const C* coef[kSet];
  const C* cpl[kSet];
  const C* top[kSet];  // dense top operators (or null)
  int sel[kSet][4];    // R_BWD0S: the rows to compute, -1 = unused
  int lo[kSet], hi[kSet];  // R_BWD0R: the rows [lo, hi) to compute
  const C* tri[kSet];  // level-0 odd blocks' tridiagonal factors [q][3][n/2] (or null)
};

template <typename C, int MODE>
__global__ __launch_bounds__(256, 4) void k_rstep(SlabSet<C> S, size_t o0, size_t o1, size_t o2, int n, int q,
                                              int nl, int shift, int RS) {
  __shared__ C xs[3 * kMaxQ];
  __shared__ C part[256];
  const int z = blockIdx.y;
  const C* __restrict__ g = S.g[z];
  C* __restrict__ t = S.t[z];
  C* __restrict__ y = S.y[z];
  const C* __restrict__ m0 = S.fac[z] + o0;
  const C* __restrict__ m1 = S.fac[z] + o1;
  const C* __restrict__ m2 = S.fac[z] + o2;
  // the RS row tiles of a block on one XCD: they share the 128-byte lines
  // that straddle tile boundaries through that XCD's L2
  const int lid = bstep_remap(blockIdx.x, gridDim.x);
  const int blk = lid / RS, rs = lid % RS;
  const int rlo = MODE == R_BWD0R ? S.lo[z] : 0, rhi = MODE == R_BWD0R ? S.hi[z] : q;
  const int R = MODE == R_BWD0S ? 4 : (rhi - rlo + RS - 1) / RS, r0 = rlo + rs * R;
  const int tid = threadIdx.x;
  const int rl = tid % R, grp = tid / R, G = 256 / R;
  // row of tile entry i: r0 + i, or the selected row (R_BWD0S; the four
  // rows read as uniform values and picked per lane by selects, not by a
  // per-lane index into the argument array, which would go through scratch)
  const int s0 = MODE == R_BWD0S ? S.sel[z][0] : 0, s1 = MODE == R_BWD0S ? S.sel[z][1] : 0;
  const int s2 = MODE == R_BWD0S ? S.sel[z][2] : 0, s3 = MODE == R_BWD0S ? S.sel[z][3] : 0;
  auto row_of = [&](int i) {
    return MODE == R_BWD0S ? (i == 0 ? s0 : (i == 1 ? s1 : (i == 2 ? s2 : s3))) : r0 + i;
  };
  const bool act = grp < G && (MODE == R_BWD0S ? row_of(rl) >= 0 : r0 + rl < rhi);
  const size_t qq = (size_t)q * q;
  int k = 0, T = 1;
  bool hm = false;
  const C* M0 = nullptr;
  const C* M1 = nullptr;
  const C* M2 = nullptr;
  if (MODE == R_ODD0 || MODE == R_BWD0 || MODE == R_BWD0S || MODE == R_BWD0R || MODE == R_ODDL) {
    k = 2 * blk + 1;
    M0 = m0 + blk * qq;
  } else if (MODE == R_FWD) {
    k = 2 * blk;
    hm = k >= 1;
    const bool hp = k + 1 < nl;
    T = (int)hm + (int)hp;
    M0 = hm ? m0 + blk * qq : m1 + blk * qq;
    M1 = m1 + blk * qq;
  } else if (MODE == R_LAST) {
    M0 = m0;
  } else {  // R_BWD
    k = 2 * blk + 1;
    T = k + 1 < nl ? 3 : 2;
    M0 = m0 + blk * qq;
    M1 = m1 + blk * qq;
    M2 = m2 + blk * qq;
  }
  const int V = T * q;
  // factor elements first: every load of this thread in flight at once
  constexpr int NC = RCols<MODE>::N;
  C mv[NC];
#pragma unroll
  for (int j = 0; j < NC; ++j) {
    const int v = grp + G * j;
    mv[j] = tmk<C>(0, 0);
    if (act && v < V) {
      const int tt = v >= 2 * q ? 2 : (v >= q ? 1 : 0);
      const C* Mt = tt == 0 ? M0 : (tt == 1 ? M1 : M2);
      mv[j] = Mt[(size_t)(v - tt * q) * q + row_of(rl)];
    }
  }
  // inputs x_t (flat over the T*q virtual columns)
  for (int e = tid; e < V; e += 256) {
    const int tt = e >= 2 * q ? 2 : (e >= q ? 1 : 0), c = e - tt * q;
    C v;
    if (MODE == R_ODD0) {
      v = g[(size_t)k * q + c];
    } else if (MODE == R_FWD) {
      const int row = (tt == 0 && hm) ? k - 1 : k + 1;
      v = t[((size_t)row << shift) * q + c];
    } else if (MODE == R_LAST) {
      v = t[c];
    } else if (MODE == R_BWD) {
      if (tt == 0) v = t[((size_t)k << shift) * q + c];
      else v = tneg(y[((size_t)(tt == 1 ? k - 1 : k + 1) << shift) * q + c]);
    } else if (MODE == R_ODDL) {
      v = t[((size_t)k << shift) * q + c];
    } else {  // R_BWD0: L_k y_{k-1} + U_k y_{k+1}, formed by k_odd0_lu in t's odd rows
      v = t[(size_t)k * q + c];
    }
    xs[e] = v;
  }
  __syncthreads();
  C acc = tmk<C>(0, 0);
#pragma unroll
  for (int j = 0; j < NC; ++j) acc = tfma(mv[j], xs[min(grp + G * j, V - 1)], acc);
  part[tid] = acc;  // part[grp * R + rl]
  __syncthreads();
  if (tid < R && (MODE == R_BWD0S ? row_of(tid) >= 0 : r0 + tid < rhi)) {
    C sum = tmk<C>(0, 0);
#pragma unroll 8
    for (int gg = 0; gg < G; ++gg) sum = tadd(sum, part[gg * R + tid]);
    const int r = row_of(tid);
    if (MODE == R_ODD0) y[(size_t)k * q + r] = sum;
    else if (MODE == R_FWD) { C* o = t + ((size_t)k << shift) * q + r; *o = tsub(*o, sum); }
    else if (MODE == R_LAST) y[r] = sum;
    else if (MODE == R_BWD || MODE == R_ODDL) y[((size_t)k << shift) * q + r] = sum;
    else { C* o = y + (size_t)k * q + r; *o = tsub(*o, sum); }
  }
}

// Level 0, odd blocks, as tridiagonal systems.  The diagonal block D_k of a
// level-0 odd block k couples each point of grid column k only to the
// points above and below it (the 9-point stencil's vertical neighbours), so
// D_k is tridiagonal and D_k x = b needs three numbers per row instead of
// the q x q inverse.  One wave solves one block by parallel cyclic
// reduction (no pivoting): lane L holds rows L and L + 64 (q <= 128); each
// of the ceil(log2 q) steps eliminates, from every row, its couplings to the
// rows s above and below (s = 1, 2, 4, ...), until every row stands alone.
// The sub-diagonal, diagonal and super-diagonal of every block are kept as
// [n/2][3][q] (zero sub- and super-diagonal outside the block).  The plan
// compares every block's reduction with its dense inverse and keeps the
// dense steps when one disagrees.  blockIdx.x the block, blockIdx.y the slab.
constexpr int kPcrRows = 128;

// 1 / x from the hardware reciprocal estimate refined by Newton-Raphson
// steps r <- r + r (1 - x r) (two in FP64, one in FP32: each doubles the
// correct bits), about one ulp, in place of a full IEEE division.
__device__ __forceinline__ double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  return fma(r, fma(-x, r, 1.0), r);
}
__device__ __forceinline__ float rcp_nr(float x) {
  const float r = __builtin_amdgcn_rcpf(x);
  return fmaf(r, fmaf(-x, r, 1.f), r);
}
template <typename C>
__device__ __forceinline__ C trcp(C b) {  // 1 / b = conj(b) / |b|^2
  const auto r = rcp_nr(fma(b.x, b.x, b.y * b.y));
  C o;
  o.x = b.x * r;
  o.y = -b.y * r;
  return o;
}

// Every row publishes the reciprocal of its own diagonal entry once per
// step, so the rows s above and below it multiply instead of dividing.
template <typename C>
__device__ __forceinline__ void pcr_wave(const C* __restrict__ abc, C (&d)[2], int q, C* __restrict__ sh) {
  const int lane = threadIdx.x;
  C* sa = sh;
  C* sr = sh + kPcrRows;
  C* sc = sh + 2 * kPcrRows;
  C* sd = sh + 3 * kPcrRows;
  C a[2], b[2], c[2];
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int i = lane + 64 * u;
    const bool in = i < q;
    a[u] = in ? abc[i] : tmk<C>(0, 0);
    b[u] = in ? abc[q + i] : tmk<C>(1, 0);
    c[u] = in ? abc[2 * q + i] : tmk<C>(0, 0);
    if (!in) d[u] = tmk<C>(0, 0);
  }
  for (int s = 1; s < q; s <<= 1) {
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int i = lane + 64 * u;
      if (i < q) {
        sa[i] = a[u];
        sr[i] = trcp(b[u]);
        sc[i] = c[u];
        sd[i] = d[u];
      }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int i = lane + 64 * u;
      if (i >= q) continue;
      C na = tmk<C>(0, 0), nc = tmk<C>(0, 0), nb = b[u], nd = d[u];
      if (i - s >= 0) {  // alpha = -a_i / b_{i-s}
        const C al = tneg(tmul(a[u], sr[i - s]));
        na = tmul(al, sa[i - s]);
        nb = tfma(al, sc[i - s], nb);
        nd = tfma(al, sd[i - s], nd);
      }
      if (i + s < q) {  // gamma = -c_i / b_{i+s}
        const C ga = tneg(tmul(c[u], sr[i + s]));
        nc = tmul(ga, sc[i + s]);
        nb = tfma(ga, sa[i + s], nb);
        nd = tfma(ga, sd[i + s], nd);
      }
      a[u] = na;
      b[u] = nb;
      c[u] = nc;
      d[u] = nd;
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < 2; ++u) d[u] = tmul(d[u], trcp(b[u]));
}

// y_k = D_k^{-1} g_k (the level-0 odd step).
template <typename C>
__global__ __launch_bounds__(64) void k_tri_odd0(SlabSet<C> S, int n, int q) {
  __shared__ C sh[4 * kPcrRows];
  const int z = blockIdx.y, j = blockIdx.x, k = 2 * j + 1, lane = threadIdx.x;
  const C* __restrict__ g = S.g[z] + (size_t)k * q;
  C d[2];
#pragma unroll
  for (int u = 0; u < 2; ++u) d[u] = lane + 64 * u < q ? g[lane + 64 * u] : tmk<C>(0, 0);
  pcr_wave<C>(S.tri[z] + (size_t)j * 3 * q, d, q, sh);
  C* __restrict__ y = S.y[z] + (size_t)k * q;
#pragma unroll
  for (int u = 0; u < 2; ++u)
    if (lane + 64 * u < q) y[lane + 64 * u] = d[u];
}

// y_k -= D_k^{-1} t_k on the rows the step completes (all of them, the rows
// S.sel, or [S.lo, S.hi)), t_k = L_k y_{k-1} + U_k y_{k+1} as formed by
// k_odd0_lu.
template <typename C, int ROWS>
__global__ __launch_bounds__(64) void k_tri_bwd0(SlabSet<C> S, int n, int q) {
  __shared__ C sh[4 * kPcrRows];
  const int z = blockIdx.y, j = blockIdx.x, k = 2 * j + 1, lane = threadIdx.x;
  const C* __restrict__ t = S.t[z] + (size_t)k * q;
  C d[2];
#pragma unroll
  for (int u = 0; u < 2; ++u) d[u] = lane + 64 * u < q ? t[lane + 64 * u] : tmk<C>(0, 0);
  pcr_wave<C>(S.tri[z] + (size_t)j * 3 * q, d, q, sh);
  const int s0 = S.sel[z][0], s1 = S.sel[z][1], s2 = S.sel[z][2], s3 = S.sel[z][3];
  const int lo = S.lo[z], hi = S.hi[z];
  C* __restrict__ y = S.y[z] + (size_t)k * q;
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int r = lane + 64 * u;
    bool keep = r < q;
    if (ROWS == 1) keep = keep && (r == s0 || r == s1 || r == s2 || r == s3);
    if (ROWS == 2) keep = keep && r >= lo && r < hi;
    if (keep) y[r] = tsub(y[r], d[u]);
  }
}

// Level 1 through the tridiagonal level-0 blocks.  Eliminating the odd
// level-0 blocks couples level-0 block k to k - 2 by L'_k = -L_k D_{k-1}^{-1}
// L_{k-1} and to k + 2 by U'_k = -U_k D_{k+1}^{-1} U_{k+1}, products of
// tridiagonal blocks and the inverse of a tridiagonal one: they are applied
// as two tridiagonal products around a tridiagonal solve instead of being
// stored dense.  The level-1 forward step t_k -= L'_k z_{k-2} + U'_k z_{k+2}
// (z = D'^{-1} t at the odd level-1 blocks, left in y by R_ODDL) and the
// backward step's right-hand side t_k - L'_k y_{k-2} - U'_k y_{k+2} are both
// t_k += L_k D_{k-1}^{-1} L_{k-1} y_{k-2} + U_k D_{k+1}^{-1} U_{k+1} y_{k+2}
// on the level-0 blocks k = k0, k0 + 4, ... (k0 = 0: the even level-1
// blocks, 2: the odd ones).  One wave per block k, blockIdx.y the slab.
template <typename C>
__global__ __launch_bounds__(64) void k_l1_couple(SlabSet<C> S, int n, int q, int k0) {
  __shared__ C sh[4 * kPcrRows];
  __shared__ C sv[kPcrRows];
  const int z = blockIdx.y, lane = threadIdx.x, k = k0 + 4 * blockIdx.x;
  if (k >= n) return;  // the whole workgroup
  const C* __restrict__ y = S.y[z];
  const C* __restrict__ cpl = S.cpl[z];
  C acc[2] = {tmk<C>(0, 0), tmk<C>(0, 0)};
  for (int side = 0; side < 2; ++side) {
    const int km = side ? k + 1 : k - 1, ks = side ? k + 2 : k - 2;
    if (ks < 0 || ks >= n) continue;  // uniform
    // w = (km's coupling towards ks) y_ks
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int r = lane + 64 * u;
      if (r < q) sv[r] = y[(size_t)ks * q + r];
    }
    __syncthreads();
    C d[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int r = lane + 64 * u;
      C w = tmk<C>(0, 0);
      if (r < q) {
        const C* cp = cpl + (size_t)km * 6 * q + side * q + r;
        for (int dZ = -1; dZ <= 1; ++dZ) {
          const int rr = r + dZ;
          if (rr >= 0 && rr < q) w = tfma(cp[(size_t)(2 * (dZ + 1)) * q], sv[rr], w);
        }
      }
      d[u] = w;
    }
    // x = D_km^{-1} w (km odd)
    pcr_wave<C>(S.tri[z] + (size_t)((km - 1) / 2) * 3 * q, d, q, sh);
    // acc += (k's coupling towards km) x (every lane done reading sv first)
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int r = lane + 64 * u;
      if (r < q) sv[r] = d[u];
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int r = lane + 64 * u;
      if (r >= q) continue;
      const C* cp = cpl + (size_t)k * 6 * q + side * q + r;
      for (int dZ = -1; dZ <= 1; ++dZ) {
        const int rr = r + dZ;
        if (rr >= 0 && rr < q) acc[u] = tfma(cp[(size_t)(2 * (dZ + 1)) * q], sv[rr], acc[u]);
      }
    }
    __syncthreads();
  }
  C* __restrict__ t = S.t[z] + (size_t)k * q;
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int r = lane + 64 * u;
    if (r < q) t[r] = tadd(t[r], acc[u]);
  }
}

// The three diagonals of every level-0 odd block of a slab from its
// assembled stencil, in the type T of the solves.
template <typename T>
__global__ void k_tri_coef(const cplx* __restrict__ coef, T* __restrict__ tri, int n, int q) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (size_t)(n / 2) * q) return;
  const int j = (int)(e / q), r = (int)(e % q), k = 2 * j + 1;
  const cplx* cf = coef + ((size_t)k * q + r) * 9;
  const cplx a = r > 0 ? cf[1] : cmk(0, 0), b = cf[4], c = r + 1 < q ? cf[7] : cmk(0, 0);
  T* o = tri + (size_t)j * 3 * q + r;
  o[0] = tmk<T>(a.x, a.y);
  o[q] = tmk<T>(b.x, b.y);
  o[2 * q] = tmk<T>(c.x, c.y);
}

// Largest relative difference, over the level-0 odd blocks of a slab,
// between the reduction's D_k^{-1} e and the dense inverse's Dinv_k e (e =
// all ones; FP64), as the bits of a non-negative float (atomicMax on the
// bits orders them as the values).
__global__ __launch_bounds__(64) void k_tri_check(const cplx* __restrict__ tri, const cplx* __restrict__ dinv,
                                                  int n, int q, unsigned* __restrict__ worst) {
  __shared__ cplx sh[4 * kPcrRows];
  __shared__ double red[2][64];
  const int j = blockIdx.x, lane = threadIdx.x;
  cplx d[2] = {cmk(1, 0), cmk(1, 0)};
  pcr_wave<cplx>(tri + (size_t)j * 3 * q, d, q, sh);
  const cplx* D = dinv + (size_t)j * q * q;
  double num = 0.0, den = 0.0;
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int r = lane + 64 * u;
    if (r >= q) continue;
    cplx e = cmk(0, 0);
    for (int c = 0; c < q; ++c) e = tadd(e, D[(size_t)c * q + r]);
    const double ex = d[u].x - e.x, ey = d[u].y - e.y;
    num = fmax(num, sqrt(ex * ex + ey * ey));
    den = fmax(den, sqrt(e.x * e.x + e.y * e.y));
  }
  red[0][lane] = num;
  red[1][lane] = den;
  __syncthreads();
  if (lane == 0) {
    for (int l = 1; l < 64; ++l) {
      num = fmax(num, red[0][l]);
      den = fmax(den, red[1][l]);
    }
    const float rel = den > 0.0 ? (float)(num / den) : (num > 0.0 ? 1e30f : 0.0f);
    atomicMax(worst, __float_as_uint(isfinite(rel) ? rel : 1e30f));
  }
}

// level 0, odd blocks: t_k = L_k y_{k-1} + U_k y_{k+1} (L, U from the
// coupling table; the odd rows of t are free once the forward elimination
// is done).  One thread per row of an odd block, blockIdx.y the slab.
template <typename C>
__global__ __launch_bounds__(256) void k_odd0_lu(SlabSet<C> S, int n, int q) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (n / 2) * q) return;
  const int j = e / q, r = e - j * q, k = 2 * j + 1;
  const C* __restrict__ y = S.y[blockIdx.y];
  C* __restrict__ t = S.t[blockIdx.y];
  const C* __restrict__ cp = S.cpl[blockIdx.y] + (size_t)k * 6 * q + r;
  C acc = tmk<C>(0, 0);
  for (int dZ = -1; dZ <= 1; ++dZ) {
    const int rr = r + dZ;
    if (rr < 0 || rr >= q) continue;
    acc = tfma(cp[(size_t)(2 * (dZ + 1)) * q], y[(size_t)(k - 1) * q + rr], acc);
    if (k + 1 < n) acc = tfma(cp[(size_t)(2 * (dZ + 1) + 1) * q], y[(size_t)(k + 1) * q + rr], acc);
  }
  t[(size_t)k * q + r] = acc;
}

// cpl[k][c][r] (type T) from coef[k][r][9]: c = 2 (dZ + 1) + side takes the
// stencil entry (dZ + 1) * 3 + 2 side (side 0: block k - 1, side 1: k + 1).
template <typename T>
__global__ void k_couplings(const cplx* __restrict__ coef, T* __restrict__ cpl, int n, int q) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (size_t)n * 6 * q) return;
  const int r = (int)(e % q);
  const size_t kc = e / q;
  const int c = (int)(kc % 6);
  const size_t k = kc / 6;
  const cplx v = coef[(k * q + r) * 9 + (c / 2) * 3 + 2 * (c & 1)];
  cpl[e] = tmk<T>(v.x, v.y);
}

// The top levels of the reduction (from level top_level, at most
// kTopBlocks blocks) as one dense operator: y_top = Top t_top on the
// Nt = nl * q unknowns of that level (rows j << top_level of the frame).
// One wave per output row streams its row of Top (all kTopK loads per lane
// in flight), the inputs sit in LDS, and the row sum is a wave reduction.
constexpr int kTopBlocks = 16;
constexpr int kTopK = 24;                 // ceil(kTopBlocks * kMaxQ / 64)
constexpr int kTopMax = kTopBlocks * kMaxQ;
constexpr int kTopBatchMin = 16;  // right-hand sides from which batched solves use the top operator
// Plans with the decoupled sweep and fewer right-hand sides run their slabs
// as multi-slab launches, where the narrow levels are no longer latency
// bound but the dense operator's bytes are streamed: there the operator
// starts at 8 blocks (one more reduction level, a quarter of the bytes).
constexpr int kTopBlocksDec = 8;

template <typename C>
__global__ __launch_bounds__(256) void k_top(SlabSet<C> S, int Nt, int q, int shift) {
  __shared__ C tv[kTopMax];
  const C* __restrict__ top = S.top[blockIdx.y];
  const C* __restrict__ t = S.t[blockIdx.y];
  C* __restrict__ y = S.y[blockIdx.y];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int o = blockIdx.x * 4 + w;
  C mv[kTopK];
#pragma unroll
  for (int k = 0; k < kTopK; ++k) {
    const int b = lane + 64 * k;
    mv[k] = (o < Nt && b < Nt) ? top[(size_t)o * Nt + b] : tmk<C>(0, 0);
  }
  // the inputs: every load issued before the first LDS store
  constexpr int TE = (kTopMax + 255) / 256;
  C tin[TE];
#pragma unroll
  for (int u = 0; u < TE; ++u) {
    const int e = threadIdx.x + 256 * u;
    const int j = e / q, r = e - j * q;
    tin[u] = e < Nt ? t[((size_t)j << shift) * q + r] : tmk<C>(0, 0);
  }
#pragma unroll
  for (int u = 0; u < TE; ++u) {
    const int e = threadIdx.x + 256 * u;
    if (e < Nt) tv[e] = tin[u];
  }
  __syncthreads();
  C acc = tmk<C>(0, 0);
#pragma unroll
  for (int k = 0; k < kTopK; ++k) acc = tfma(mv[k], tv[min(lane + 64 * k, Nt - 1)], acc);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    acc.x += __shfl_xor(acc.x, off);
    acc.y += __shfl_xor(acc.y, off);
  }
  if (lane == 0 && o < Nt) {
    const int j = o / q, r = o - j * q;
    y[((size_t)j << shift) * q + r] = acc;
  }
}

// x[b][b] = 1, 0 elsewhere (Nt x Nt)
__global__ void k_identity(cplx* __restrict__ x, int Nt) {
  const size_t cnt = (size_t)Nt * Nt;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < cnt; e += (size_t)gridDim.x * blockDim.x)
    x[e] = cmk(e / Nt == e % Nt ? 1.0 : 0.0, 0.0);
}

// out[o][b] = in[b][o] (rounded to the storage type)
template <typename T>
__global__ void k_transpose_to(const cplx* __restrict__ in, T* __restrict__ out, int Nt) {
  const size_t cnt = (size_t)Nt * Nt;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < cnt; e += (size_t)gridDim.x * blockDim.x) {
    const size_t o = e / Nt, b = e % Nt;
    const cplx v = in[b * Nt + o];
    out[e] = tmk<T>(v.x, v.y);
  }
}

// level 0, even blocks: t_k = g_k - L_k z_{k-1} - U_k z_{k+1} with z_j = y_j
template <typename C>
__global__ __launch_bounds__(256) void k_even0(SlabSet<C> S, int n, int q) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ((n + 1) / 2) * q) return;
  const int j = e / q, r = e - j * q, k = 2 * j;
  const C* __restrict__ g = S.g[blockIdx.y];
  const C* __restrict__ y = S.y[blockIdx.y];
  C* __restrict__ t = S.t[blockIdx.y];
  const C* __restrict__ cp = S.cpl[blockIdx.y] + (size_t)k * 6 * q + r;
  C acc = g[(size_t)k * q + r];
  for (int dZ = -1; dZ <= 1; ++dZ) {
    const int rr = r + dZ;
    if (rr < 0 || rr >= q) continue;
    if (k >= 1) acc = tsub(acc, tmul(cp[(size_t)(2 * (dZ + 1)) * q], y[(size_t)(k - 1) * q + rr]));
    if (k + 1 < n) acc = tsub(acc, tmul(cp[(size_t)(2 * (dZ + 1) + 1) * q], y[(size_t)(k + 1) * q + rr]));
  }
  t[(size_t)k * q + r] = acc;
}

// ---------------------------------------------------------------- batched
// The same level steps for B right-hand sides x[b][n][q] (stride xs_b):
// y = sum_t M_t X_t with q x q factor blocks M_t and q x BT right-hand-side
// panels X_t.  A workgroup of NT threads takes one block and a tile of BT
// right-hand sides.  It stages the panels in LDS (coalesced along the
// block's rows), then thread (r, g) = (tid % q, tid / q) multiplies row r of
// the columns c = g, g + G, ... (G = NT / q groups) into BT accumulators:
// every factor element is loaded once per tile, straight from memory into a
// register (U loads in flight per thread), and the G partial sums are added
// through LDS.  Three tile shapes trade factor re-reads (B / BT per block)
// against parallelism on the upper levels, where there are few blocks.
enum { BSTEP_FWD = 0, BSTEP_BWD = 1, BSTEP_LAST = 2, BSTEP_ODD0 = 3, BSTEP_BWD0 = 4 };
template <typename C, int BT, int NT>
struct BShape {
  static constexpr int XS = BT + 16 / (int)sizeof(C);  // padded panel row (complex entries)
  static constexpr int U = 4;                           // factor loads in flight per thread
  static constexpr int ROWS = (3 * kMaxQ > NT) ? 3 * kMaxQ : NT;
  static constexpr size_t lds() { return (size_t)ROWS * XS * sizeof(C); }
};
// tile variants: index 0 widest (most right-hand sides per workgroup)
template <typename C> struct BVariants;
template <> struct BVariants<fcplx> {
  static constexpr int BT[3] = {16, 8, 4};
  static constexpr int NT[3] = {256, 512, 1024};
};
template <> struct BVariants<cplx> {
  static constexpr int BT[3] = {8, 4, 2};
  static constexpr int NT[3] = {256, 512, 1024};
};

template <typename C, int MODE, int BT, int NT>
__global__ __launch_bounds__(NT) void k_bstep(C* __restrict__ x, size_t xs_b, int B,
                                              const C* __restrict__ m0, const C* __restrict__ m1,
                                              const C* __restrict__ m2,
                                              const C* __restrict__ coef, int n, int q, int nl,
                                              int shift, int tiles, int total) {
  using S = BShape<C, BT, NT>;
  constexpr int XS = S::XS, U = S::U;
  extern __shared__ unsigned char lds_raw[];
  C* xs = reinterpret_cast<C*>(lds_raw);  // panels [t][c][XS], later partial sums [g][r][XS]
  const int lid = bstep_remap(blockIdx.x, total);
  const int blk = lid / tiles;
  const int b0 = (lid % tiles) * BT;
  const int nbt = min(BT, B - b0);
  const size_t qq = (size_t)q * q;
  const int tid = threadIdx.x;
  // panel rows (global row index, sign) and factor blocks per mode
  int T = 0, k = 0;
  int row[3] = {0, 0, 0};
  bool neg[3] = {false, false, false};
  const C* M[3] = {nullptr, nullptr, nullptr};
  if (MODE == BSTEP_FWD) {
    k = 2 * blk;
    if (k >= 1) { row[T] = (k - 1) << shift; M[T++] = m0 + blk * qq; }
    if (k + 1 < nl) { row[T] = (k + 1) << shift; M[T++] = m1 + blk * qq; }
  } else if (MODE == BSTEP_BWD) {
    k = 2 * blk + 1;
    row[0] = k << shift; M[0] = m0 + blk * qq;
    row[1] = (k - 1) << shift; neg[1] = true; M[1] = m1 + blk * qq;
    T = 2;
    if (k + 1 < nl) { row[2] = (k + 1) << shift; neg[2] = true; M[2] = m2 + blk * qq; T = 3; }
  } else if (MODE == BSTEP_LAST) {
    k = 0; row[0] = 0; M[0] = m0; T = 1;
  } else {  // ODD0, BWD0 (level 0)
    k = 2 * blk + 1; row[0] = k; M[0] = m0 + blk * qq; T = 1;
  }
  // Thread (r, g) = (tid % q, tid / q): row r of the factor columns g,
  // g + G, ... (G = NT / q groups), and column r of the panel pairs
  // (panel t, right-hand side bb) = slot g, g + G, ... when staging.
  const int G = NT / q;
  const int r = tid % q, g = tid / q;
  const bool act = g < G;
  const int per_t = q * nbt;
  // factor chunk (t, c0): columns c0 + u G of M_t, U loads in flight; the
  // first chunk's loads go out before the staging
  C cur[U];
  int ft = 0, fc = g;
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int c = fc + u * G;
    cur[u] = act && T > 0 && c < q ? M[0][(size_t)c * q + r] : tmk<C>(0, 0);
  }
  if (MODE == BSTEP_BWD0) {  // L_k x_{k-1} + U_k x_{k+1} from the stencil coefficients
    for (int e = tid; e < per_t; e += NT) {
      const int bb = e / q, c = e - bb * q;
      const C* xb = x + (size_t)(b0 + bb) * xs_b;
      const C* cf = coef + ((size_t)k * q + c) * 9;
      C v = tmk<C>(0, 0);
      for (int dZ = -1; dZ <= 1; ++dZ) {
        const int rr = c + dZ;
        if (rr < 0 || rr >= q) continue;
        v = tfma(cf[(dZ + 1) * 3 + 0], xb[(size_t)(k - 1) * q + rr], v);
        if (k + 1 < n) v = tfma(cf[(dZ + 1) * 3 + 2], xb[(size_t)(k + 1) * q + rr], v);
      }
      xs[(size_t)c * XS + bb] = v;
    }
    for (int e = tid; e < q * (BT - nbt); e += NT)  // unused right-hand-side slots
      xs[(size_t)(e / (BT - nbt)) * XS + nbt + e % (BT - nbt)] = tmk<C>(0, 0);
  } else {
    // pairs pr = t BT + bb (zero for bb >= nbt); at most EPT per thread since
    // G >= NT / kMaxQ; every load issued before the stores
    constexpr int EPT = (3 * BT + NT / kMaxQ - 1) / (NT / kMaxQ);
    C sv[EPT];
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const int pr = g + i * G, t = pr / BT, bb = pr % BT;
      sv[i] = tmk<C>(0, 0);
      if (act && t < T && bb < nbt) {
        const int rw = t == 0 ? row[0] : (t == 1 ? row[1] : row[2]);
        sv[i] = x[(size_t)(b0 + bb) * xs_b + (size_t)rw * q + r];
        if ((t == 0 ? neg[0] : (t == 1 ? neg[1] : neg[2]))) sv[i] = tneg(sv[i]);
      }
    }
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const int pr = g + i * G, t = pr / BT, bb = pr % BT;
      if (act && t < T) xs[((size_t)t * kMaxQ + r) * XS + bb] = sv[i];
    }
  }
  __syncthreads();
  C acc[BT];
#pragma unroll
  for (int j = 0; j < BT; ++j) acc[j] = tmk<C>(0, 0);
  if (act) {
    while (ft < T) {
      // the next chunk's loads go out before this chunk's products
      int nt = ft, nc = fc + U * G;
      if (nc >= q) {
        nt = ft + 1;
        nc = g;
      }
      C nxt[U];
      const C* Mn = nt == 1 ? M[1] : (nt == 2 ? M[2] : M[0]);
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int c = nc + u * G;
        nxt[u] = nt < T && c < q ? Mn[(size_t)c * q + r] : tmk<C>(0, 0);
      }
      const C* Xt = xs + (size_t)ft * kMaxQ * XS;
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int c = min(fc + u * G, q - 1);  // cur is zero past the end
        const C* xr = Xt + (size_t)c * XS;
#pragma unroll
        for (int j = 0; j < BT; ++j) acc[j] = tfma(cur[u], xr[j], acc[j]);
      }
#pragma unroll
      for (int u = 0; u < U; ++u) cur[u] = nxt[u];
      ft = nt;
      fc = nc;
    }
  }
  __syncthreads();  // panels consumed; reuse LDS for the partial sums
  if (act) {
#pragma unroll
    for (int j = 0; j < BT; ++j) xs[(size_t)tid * XS + j] = acc[j];
  }
  __syncthreads();
  const size_t okq = (size_t)(MODE == BSTEP_FWD || MODE == BSTEP_BWD ? (k << shift) : k) * q;
  if (act) {
    for (int bb = g; bb < nbt; bb += G) {
      C sum = tmk<C>(0, 0);
      for (int gg = 0; gg < G; ++gg) sum = tadd(sum, xs[(size_t)(gg * q + r) * XS + bb]);
      C* o = x + (size_t)(b0 + bb) * xs_b + okq + r;
      if (MODE == BSTEP_FWD || MODE == BSTEP_BWD0)
        *o = tsub(*o, sum);
      else
        *o = sum;
    }
  }
}

// FP32 batched level step on matrix cores (v_mfma_f32_16x16x4f32): the
// same y = sum_t M_t X_t as k_bstep for a tile of kMB right-hand sides.
// Wave w owns output rows [16 w, 16 w + 16) of the block for all kMB
// right-hand sides (two 16-column tiles).  The panels X_t are staged in LDS
// as real and imaginary planes; each K step of 4 factor columns feeds one
// factor element per lane (lane l: row 16 w + l % 16, column l / 16, read
// straight from memory, U steps in flight) and 4 real MFMAs per complex
// 16 x 16 x 4 product: Re += Ar Br - Ai Bi, Im += Ar Bi + Ai Br.
constexpr int kMB = 32;
typedef float f32x4_t __attribute__((ext_vector_type(4)));

__host__ __device__ constexpr int mq4(int q) { return (q + 3) & ~3; }
// panels staged per mode: 3 (backward), 2 (forward) or 1
template <int MODE>
__host__ __device__ constexpr int bstep_panels() { return MODE == BSTEP_BWD ? 3 : (MODE == BSTEP_FWD ? 2 : 1); }
template <int MODE>
inline size_t bstep_mfma_lds(int q) { return (size_t)2 * bstep_panels<MODE>() * mq4(q) * (kMB + 1) * sizeof(float); }

// Factor element of K step s for lane (row ra, column kk of the step):
// panel t = s / KS, column 4 (s % KS) + kk of M_t; zero past the end.
__device__ __forceinline__ fcplx bstep_fac(const fcplx* M0, const fcplx* M1, const fcplx* M2, int s, int S,
                                           int KS, int kk, int q, bool rin, int ra) {
  const int t = s >= 2 * KS ? 2 : (s >= KS ? 1 : 0);
  const int c = 4 * (s - t * KS) + kk;
  const fcplx* Mt = t == 0 ? M0 : (t == 1 ? M1 : M2);
  return (s < S && c < q && rin) ? Mt[(size_t)c * q + ra] : tmk<fcplx>(0, 0);
}

template <int MODE>
__global__ __launch_bounds__(384) void k_bstep_mfma(fcplx* __restrict__ x, size_t xs_b, int B,
                                                    const fcplx* __restrict__ m0, const fcplx* __restrict__ m1,
                                                    const fcplx* __restrict__ m2, const fcplx* __restrict__ coef,
                                                    int n, int q, int nl, int shift, int tiles, int total) {
  constexpr int U = 4, LB = kMB + 1;  // K steps in flight; padded panel row
  extern __shared__ unsigned char lds_raw[];
  const int q4 = mq4(q);
  float* xr = reinterpret_cast<float*>(lds_raw);  // [panels][q4][LB]
  float* xi = xr + bstep_panels<MODE>() * q4 * LB;
  const int lid = bstep_remap(blockIdx.x, total);
  const int blk = lid / tiles;
  const int b0 = (lid % tiles) * kMB;
  const int nbt = min(kMB, B - b0);
  const size_t qq = (size_t)q * q;
  const int tid = threadIdx.x, NT = blockDim.x;
  // panel t: global row rw_t, negated for t >= 1 in BWD, factor block M_t
  int T = 0, k = 0, rw0 = 0, rw1 = 0, rw2 = 0;
  const fcplx* M0 = nullptr;
  const fcplx* M1 = nullptr;
  const fcplx* M2 = nullptr;
  if (MODE == BSTEP_FWD) {
    k = 2 * blk;
    const bool lo = k >= 1, hi = k + 1 < nl;
    rw0 = lo ? (k - 1) << shift : (k + 1) << shift;
    M0 = (lo ? m0 : m1) + blk * qq;
    rw1 = (k + 1) << shift;
    M1 = m1 + blk * qq;
    T = (lo ? 1 : 0) + (hi ? 1 : 0);
  } else if (MODE == BSTEP_BWD) {
    k = 2 * blk + 1;
    rw0 = k << shift; M0 = m0 + blk * qq;
    rw1 = (k - 1) << shift; M1 = m1 + blk * qq;
    rw2 = (k + 1) << shift; M2 = m2 + blk * qq;
    T = k + 1 < nl ? 3 : 2;
  } else if (MODE == BSTEP_LAST) {
    k = 0; M0 = m0; T = 1;
  } else {  // ODD0, BWD0
    k = 2 * blk + 1; rw0 = k; M0 = m0 + blk * qq; T = 1;
  }
  const int w = tid >> 6, l = tid & 63;
  const int ra = 16 * w + (l & 15);  // factor row this lane feeds
  const int kk = l >> 4;             // column within the K step
  // K steps flattened over the panels: step s is panel t = s / KS, factor
  // column c = 4 (s % KS) + kk, LDS panel row t q4 + c = 4 s + kk
  const int KS = q4 >> 2, S = T * KS;
  const bool rin = ra < q;
  // the first U steps' factor elements are in flight during the staging
  fcplx cur[U];
#pragma unroll
  for (int u = 0; u < U; ++u) cur[u] = bstep_fac(M0, M1, M2, u, S, KS, kk, q, rin, ra);
  // panels: thread (c, slot) = (tid % q4, tid / q4) stages column c of the
  // (panel, right-hand side) pairs slot, slot + SL, ... (SL = NT / q4 >= 4
  // since NT = 64 ceil(q / 16) and q4 <= 16 ceil(q / 16), so at most 8 pairs
  // per thread and panel); zero past q and past nbt
  const int c = tid % q4, slot = tid / q4, SL = NT / q4;
  const bool cact = slot < SL;
  constexpr int EPT = 8 * bstep_panels<MODE>();
  if constexpr (MODE == BSTEP_BWD0) {
    // one panel: L_k x_{k-1} + U_k x_{k+1} from the stencil coefficients.
    // Rows k - 1 and k + 1 of the pairs are loaded at once and pass through
    // the panel one after the other; each thread keeps its column's six
    // coefficients in registers and its sums until the panel is free.
    const bool hp = k + 1 < n;
    fcplx cl[3], cu[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const int rr = c + d - 1;
      const bool ok = cact && c < q && rr >= 0 && rr < q;
      const fcplx* cf = coef + ((size_t)k * q + (ok ? c : 0)) * 9;
      cl[d] = ok ? cf[d * 3 + 0] : tmk<fcplx>(0, 0);
      cu[d] = ok && hp ? cf[d * 3 + 2] : tmk<fcplx>(0, 0);
    }
    fcplx xm[EPT], xp[EPT];
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const int bb = slot + i * SL;
      const bool ld = cact && bb < nbt && c < q;
      const fcplx* xb = x + (size_t)(b0 + (ld ? bb : 0)) * xs_b + c;
      xm[i] = ld ? xb[(size_t)(k - 1) * q] : tmk<fcplx>(0, 0);
      xp[i] = ld && hp ? xb[(size_t)(k + 1) * q] : tmk<fcplx>(0, 0);
    }
    fcplx v[EPT];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      if (h) __syncthreads();  // the first row's sums are formed
#pragma unroll
      for (int i = 0; i < EPT; ++i) {
        const int bb = slot + i * SL;
        if (cact && bb < kMB) {
          xr[c * LB + bb] = h ? xp[i].x : xm[i].x;
          xi[c * LB + bb] = h ? xp[i].y : xm[i].y;
        }
      }
      __syncthreads();
#pragma unroll
      for (int i = 0; i < EPT; ++i) {
        const int bb = slot + i * SL;
        if (!h) v[i] = tmk<fcplx>(0, 0);
        if (cact && bb < kMB) {
#pragma unroll
          for (int d = 0; d < 3; ++d) {
            const int o = min(max(c + d - 1, 0), q4 - 1) * LB + bb;
            v[i] = tfma(h ? cu[d] : cl[d], tmk<fcplx>(xr[o], xi[o]), v[i]);
          }
        }
      }
    }
    __syncthreads();  // the second row's sums are formed
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const int bb = slot + i * SL;
      if (cact && bb < kMB) {
        xr[c * LB + bb] = v[i].x;
        xi[c * LB + bb] = v[i].y;
      }
    }
  } else {
    // every load issued before the stores
    fcplx sv[EPT];
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const int pr = slot + i * SL, t = pr / kMB, bb = pr % kMB;
      sv[i] = tmk<fcplx>(0, 0);
      if (cact && t < T && bb < nbt && c < q) {
        sv[i] = x[(size_t)(b0 + bb) * xs_b + (size_t)(t == 0 ? rw0 : (t == 1 ? rw1 : rw2)) * q + c];
        if (MODE == BSTEP_BWD && t > 0) sv[i] = tneg(sv[i]);
      }
    }
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const int pr = slot + i * SL, t = pr / kMB, bb = pr % kMB;
      if (cact && t < T) {
        xr[(t * q4 + c) * LB + bb] = sv[i].x;
        xi[(t * q4 + c) * LB + bb] = sv[i].y;
      }
    }
  }
  __syncthreads();
  f32x4_t dre0 = {0, 0, 0, 0}, dim0 = {0, 0, 0, 0}, dre1 = {0, 0, 0, 0}, dim1 = {0, 0, 0, 0};
  const float* pr = xr + (l & 15);
  const float* pi = xi + (l & 15);
  for (int s0 = 0; s0 < S; s0 += U) {
    // the next U steps' loads go out before this group's products
    fcplx nxt[U];
#pragma unroll
    for (int u = 0; u < U; ++u) nxt[u] = bstep_fac(M0, M1, M2, s0 + U + u, S, KS, kk, q, rin, ra);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int st = s0 + u;
      if (st >= S) break;
      const int o = (4 * st + kk) * LB;
      const float br0 = pr[o], bi0 = pi[o], br1 = pr[o + 16], bi1 = pi[o + 16];
      const float ar = cur[u].x, ai = cur[u].y;
      dre0 = __builtin_amdgcn_mfma_f32_16x16x4f32(ar, br0, dre0, 0, 0, 0);
      dre0 = __builtin_amdgcn_mfma_f32_16x16x4f32(-ai, bi0, dre0, 0, 0, 0);
      dim0 = __builtin_amdgcn_mfma_f32_16x16x4f32(ar, bi0, dim0, 0, 0, 0);
      dim0 = __builtin_amdgcn_mfma_f32_16x16x4f32(ai, br0, dim0, 0, 0, 0);
      dre1 = __builtin_amdgcn_mfma_f32_16x16x4f32(ar, br1, dre1, 0, 0, 0);
      dre1 = __builtin_amdgcn_mfma_f32_16x16x4f32(-ai, bi1, dre1, 0, 0, 0);
      dim1 = __builtin_amdgcn_mfma_f32_16x16x4f32(ar, bi1, dim1, 0, 0, 0);
      dim1 = __builtin_amdgcn_mfma_f32_16x16x4f32(ai, br1, dim1, 0, 0, 0);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) cur[u] = nxt[u];
  }
  // D layout: lane l holds rows 4 (l / 16) + i of column l % 16
  const size_t okq = (size_t)(MODE == BSTEP_FWD || MODE == BSTEP_BWD ? (k << shift) : k) * q;
#pragma unroll
  for (int ct = 0; ct < 2; ++ct)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int r = 16 * w + 4 * (l >> 4) + i, bb = 16 * ct + (l & 15);
      if (r >= q || bb >= nbt) continue;
      const fcplx val = tmk<fcplx>(ct ? dre1[i] : dre0[i], ct ? dim1[i] : dim0[i]);
      fcplx* o = x + (size_t)(b0 + bb) * xs_b + okq + r;
      if (MODE == BSTEP_FWD || MODE == BSTEP_BWD0)
        *o = tsub(*o, val);
      else
        *o = val;
    }
}

// The top operator for many right-hand sides (FP32, matrix cores):
// Y = Top X on the Nt unknowns of the top level, X and Y in place at the
// level's rows (j << shift) of every right-hand side.  Top is read column-
// major (topT[k][o]) so that the 16 rows one K step feeds are one 128-byte
// segment.  A workgroup of 4 waves takes 64 rows (16 per wave) x 32
// right-hand sides x one K slice of kTopKL; the panel of X is staged in LDS
// once for the 4 waves.  The slices' partial products go to
// part[slice][b][o] and k_top_reduce adds them in slice order
// (deterministic).
constexpr int kTopKL = 128;  // K per slice
constexpr int kTopKC = 64;   // K rows staged in LDS at a time
constexpr int kTopSlices = (kTopMax + kTopKL - 1) / kTopKL;

__global__ __launch_bounds__(256) void k_top_mfma(const fcplx* __restrict__ topT, const fcplx* __restrict__ x,
                                                  size_t xs_b, int B, int Nt, int q, int shift,
                                                  fcplx* __restrict__ part) {
  constexpr int LB = kMB + 1;
  __shared__ float xr[kTopKC * LB], xi[kTopKC * LB];
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  const int o0 = blockIdx.x * 64 + 16 * w, b0 = blockIdx.y * kMB, sl = blockIdx.z;
  const int kb = sl * kTopKL, ke = min(Nt, kb + kTopKL);
  const int nbt = min(kMB, B - b0);
  const int ra = o0 + (l & 15), kk = l >> 4;
  f32x4_t dre0 = {0, 0, 0, 0}, dim0 = {0, 0, 0, 0}, dre1 = {0, 0, 0, 0}, dim1 = {0, 0, 0, 0};
  for (int c0 = kb; c0 < ke; c0 += kTopKC) {
    const int cn = min(kTopKC, ke - c0);
    // this chunk's factor elements first: all 16 K steps in flight
    fcplx a[kTopKC / 4];
#pragma unroll
    for (int u = 0; u < kTopKC / 4; ++u) {
      const int kr = 4 * u + kk;
      a[u] = (kr < cn && ra < Nt) ? topT[(size_t)(c0 + kr) * Nt + ra] : tmk<fcplx>(0, 0);
    }
    __syncthreads();  // the previous chunk's panel is consumed
    {
      const int kr = tid & (kTopKC - 1), bq = tid / kTopKC;  // row kr, right-hand sides 8 bq .. 8 bq + 7
      const bool kin = kr < cn;
      const int k = c0 + kr, j = kin ? k / q : 0;
      const size_t off = ((size_t)j << shift) * q + (kin ? k - j * q : 0);
#pragma unroll
      for (int e = 0; e < kMB / 4; ++e) {
        const int bb = bq * (kMB / 4) + e;
        const fcplx v = (kin && bb < nbt) ? x[(size_t)(b0 + bb) * xs_b + off] : tmk<fcplx>(0, 0);
        xr[kr * LB + bb] = v.x;
        xi[kr * LB + bb] = v.y;
      }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kTopKC / 4; ++u) {
      if (4 * u >= cn) break;
      const int o = (4 * u + kk) * LB + (l & 15);
      const float br0 = xr[o], bi0 = xi[o], br1 = xr[o + 16], bi1 = xi[o + 16];
      const float ar = a[u].x, ai = a[u].y;
      dre0 = __builtin_amdgcn_mfma_f32_16x16x4f32(ar, br0, dre0, 0, 0, 0);
      dre0 = __builtin_amdgcn_mfma_f32_16x16x4f32(-ai, bi0, dre0, 0, 0, 0);
      dim0 = __builtin_amdgcn_mfma_f32_16x16x4f32(ar, bi0, dim0, 0, 0, 0);
      dim0 = __builtin_amdgcn_mfma_f32_16x16x4f32(ai, br0, dim0, 0, 0, 0);
      dre1 = __builtin_amdgcn_mfma_f32_16x16x4f32(ar, br1, dre1, 0, 0, 0);
      dre1 = __builtin_amdgcn_mfma_f32_16x16x4f32(-ai, bi1, dre1, 0, 0, 0);
      dim1 = __builtin_amdgcn_mfma_f32_16x16x4f32(ar, bi1, dim1, 0, 0, 0);
      dim1 = __builtin_amdgcn_mfma_f32_16x16x4f32(ai, br1, dim1, 0, 0, 0);
    }
  }
  // D layout: lane l holds rows 4 (l / 16) + i of column l % 16
#pragma unroll
  for (int ct = 0; ct < 2; ++ct)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int o = o0 + 4 * (l >> 4) + i, bb = 16 * ct + (l & 15);
      if (o >= Nt || bb >= nbt) continue;
      part[((size_t)sl * B + b0 + bb) * Nt + o] = tmk<fcplx>(ct ? dre1[i] : dre0[i], ct ? dim1[i] : dim0[i]);
    }
}

// x_b at the top level's rows = sum over slices of part[slice][b][o]
__global__ void k_top_reduce(const fcplx* __restrict__ part, int slices, int Nt, int B, fcplx* __restrict__ x,
                             size_t xs_b, int q, int shift) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (size_t)Nt * B) return;
  const int b = (int)(e / Nt), o = (int)(e % Nt);
  fcplx sum = tmk<fcplx>(0, 0);
  for (int sl = 0; sl < slices; ++sl) sum = tadd(sum, part[((size_t)sl * B + b) * Nt + o]);
  const int j = o / q;
  x[(size_t)b * xs_b + ((size_t)j << shift) * q + (o - j * q)] = sum;
}

template <typename C, int RB>
__global__ void k_fwd0_even_b(C* __restrict__ x, size_t xs_b, const C* __restrict__ coef, int n,
                              int q, int B) {
  // x_k -= L_k x_{k-1} + U_k x_{k+1} for the even blocks k of level 0, RB
  // right-hand sides per thread: the stencil coefficients are loaded once,
  // and every right-hand side's inputs are loaded before the first store
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  const int k = 2 * blockIdx.y;
  if (r >= q) return;
  const int b0 = blockIdx.z * RB;
  const C* cf = coef + ((size_t)k * q + r) * 9;
  const bool lo = k >= 1, hi = k + 1 < n;
  C cl[3], cu[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int rr = r + d - 1;
    const bool in = rr >= 0 && rr < q;
    cl[d] = (in && lo) ? cf[d * 3 + 0] : tmk<C>(0, 0);
    cu[d] = (in && hi) ? cf[d * 3 + 2] : tmk<C>(0, 0);
  }
  C xk[RB], xm[RB][3], xp[RB][3];
#pragma unroll
  for (int j = 0; j < RB; ++j) {
    const bool ok = b0 + j < B;
    const C* xb = x + (size_t)(ok ? b0 + j : 0) * xs_b;
    xk[j] = ok ? xb[(size_t)k * q + r] : tmk<C>(0, 0);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const int rr = r + d - 1;
      const bool in = ok && rr >= 0 && rr < q;
      xm[j][d] = (in && lo) ? xb[(size_t)(k - 1) * q + rr] : tmk<C>(0, 0);
      xp[j][d] = (in && hi) ? xb[(size_t)(k + 1) * q + rr] : tmk<C>(0, 0);
    }
  }
#pragma unroll
  for (int j = 0; j < RB; ++j) {
    if (b0 + j >= B) break;
    C acc = xk[j];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const int rr = r + d - 1;
      if (rr < 0 || rr >= q) continue;
      if (lo) acc = tsub(acc, tmul(cl[d], xm[j][d]));
      if (hi) acc = tsub(acc, tmul(cu[d], xp[j][d]));
    }
    x[(size_t)(b0 + j) * xs_b + (size_t)k * q + r] = acc;
  }
}

// ------------------------------------------------------- sweep helpers
// Trace sources on two lines of one slab (eq. pde_GRF_real): the term
// sgn * sum_dX coef[i][rt][(dZ+1)*3 + dX+1] * src(i+dX) added to rhs[i][rt],
// src(i) = s[i*qs + rs] (+ s2[i*q2 + r2] when s2 is set).
struct Inject {
  int rt, dZ;
  double sgn;
  int qs, rs;
};

template <typename T>
__device__ __forceinline__ T inject_term(const T* __restrict__ coef, int n, int q, int i, const Inject& J,
                                         const T* __restrict__ src, const T* __restrict__ s2, int q2, int r2) {
  const T* cf = coef + ((size_t)i * q + J.rt) * 9 + (J.dZ + 1) * 3;
  T acc = tmk<T>(0, 0);
  for (int dX = -1; dX <= 1; ++dX) {
    const int ii = i + dX;
    if (ii < 0 || ii >= n) continue;
    T sv = src[(size_t)ii * J.qs + J.rs];
    if (s2) sv = tadd(sv, s2[(size_t)ii * q2 + r2]);
    acc = tfma(cf[dX + 1], sv, acc);
  }
  return tmk<T>(acc.x * J.sgn, acc.y * J.sgn);
}

// The two trace sources alone: rhs[i][A.rt] and rhs[i][B.rt] of a layer
// (row stride qr) from src (row stride qs, batch stride n qs) and s2 on
// line B (many right-hand sides run this as its own launch); rhs2, when
// set, is a second copy of rhs that receives the same sums.
template <typename T>
__global__ void k_inject(T* __restrict__ rhs, int qr, const T* __restrict__ coef, int n, Inject A, Inject Bj,
                         const T* __restrict__ src, int qs, const T* __restrict__ s2, int q2, int r2,
                         T* __restrict__ rhs2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  T* rb = rhs + (size_t)blockIdx.y * n * qr;
  const T* sb = src + (size_t)blockIdx.y * n * qs;
  const T* s2b = s2 ? s2 + (size_t)blockIdx.y * n * q2 : nullptr;
  // both lines' loads before either store
  T* oa = rb + (size_t)i * qr + A.rt;
  T* ob = rb + (size_t)i * qr + Bj.rt;
  const T ta = inject_term(coef, n, qr, i, A, sb, (const T*)nullptr, 0, 0);
  const T tb = inject_term(coef, n, qr, i, Bj, sb, s2b, q2, r2);
  const T va = tadd(*oa, ta), vb = tadd(*ob, tb);
  *oa = va;
  *ob = vb;
  if (rhs2) {
    T* r2b = rhs2 + (size_t)blockIdx.y * n * qr + (size_t)i * qr;
    r2b[A.rt] = va;
    r2b[Bj.rt] = vb;
  }
}

// dst[i][r] = g(i, z0 + r) on the layer lines [a, b], 0 elsewhere; with
// sA set, the downward sweep's two trace sources from sA (the solution of
// the layer above) are added on lines A.rt and B.rt.
template <typename T>
__global__ void k_gather(const T* __restrict__ g, T* __restrict__ dst, int n, int q, int z0,
                         int a, int b, int orient, const T* __restrict__ coef, Inject A, Inject Bj,
                         const T* __restrict__ sA, T* __restrict__ dst2) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * q) return;
  g += (size_t)blockIdx.y * n * n;
  dst += (size_t)blockIdx.y * n * q;
  int i, r;
  if (orient == 0) { r = t / n; i = t % n; } else { i = t / q; r = t % q; }
  const int Z = z0 + r;
  T v = tmk<T>(0, 0);
  if (Z >= a && Z <= b) v = (orient == 0) ? g[(size_t)Z * n + i] : g[(size_t)i * n + Z];
  if (sA) {
    const T* s = sA + (size_t)blockIdx.y * n * A.qs;
    if (r == A.rt) v = tadd(v, inject_term(coef, n, q, i, A, s, (const T*)nullptr, 0, 0));
    if (r == Bj.rt) v = tadd(v, inject_term(coef, n, q, i, Bj, s, (const T*)nullptr, 0, 0));
  }
  dst[(size_t)i * q + r] = v;
  if (dst2) dst2[(size_t)blockIdx.y * n * q + (size_t)i * q + r] = v;
}

// out(i, Z) (+)= src[i][Z - z0] for Z in [a, b] (the solution of one layer
// into the grid), and, with rhs set, the upward sweep's two trace sources
// of the next layer added to its right-hand side rhs (lines A.rt, B.rt;
// sources sA = the scattered solution, plus s2 on line B).
template <typename T>
__global__ void k_scatter(const T* __restrict__ src, T* __restrict__ out, int n, int q, int z0,
                          int a, int b, int orient, int accumulate, T* __restrict__ rhs, int qr,
                          const T* __restrict__ coef, Inject A, Inject Bj, const T* __restrict__ s2, int q2,
                          int r2) {
  const int rows = b - a + 1;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n * rows) {
    const T* sb = src + (size_t)blockIdx.y * n * q;
    T* ob = out + (size_t)blockIdx.y * n * n;
    int i, Z;
    if (orient == 0) { Z = a + t / n; i = t % n; } else { i = t / rows; Z = a + t % rows; }
    const T v = sb[(size_t)i * q + (Z - z0)];
    const size_t o = (orient == 0) ? (size_t)Z * n + i : (size_t)i * n + Z;
    ob[o] = accumulate ? tadd(ob[o], v) : v;
  }
  if (rhs && t < n) {
    T* rb = rhs + (size_t)blockIdx.y * n * qr;
    const T* sa = src + (size_t)blockIdx.y * n * q;
    const T* s2b = s2 + (size_t)blockIdx.y * n * q2;
    T* o = rb + (size_t)t * qr + A.rt;
    *o = tadd(*o, inject_term(coef, n, qr, t, A, sa, (const T*)nullptr, 0, 0));
    o = rb + (size_t)t * qr + Bj.rt;
    *o = tadd(*o, inject_term(coef, n, qr, t, Bj, sa, s2b, q2, r2));
  }
}

// ------------------------------------------------------ decoupled sweep
// The trace sources one layer receives, as a map from a trace -- two grid
// lines of n values, [2][n] -- to the layer's right-hand side: line part p
// enters slab-frame row rt[p] through the couplings of stencil row dZ[p] of
// the layer's own matrix, times sgn[p] (the injections of k_gather /
// k_scatter, Section 3.2 eq. pde_GRF_real).
struct TraceInj {
  int rt[2], dZ[2];
  double sgn[2];
};

// Right-hand side of the unit trace j0 + b in x_b (b < B; x zeroed before).
__global__ void k_unit_rhs(cplx* __restrict__ x, const cplx* __restrict__ coef, int n, int q, TraceInj E,
                           int j0, int B) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  const int j = j0 + b, p = j / n, i0 = j % n;
  cplx* xb = x + (size_t)b * n * q;
  for (int i = max(i0 - 1, 0); i <= min(i0 + 1, n - 1); ++i) {
    const cplx c = coef[((size_t)i * q + E.rt[p]) * 9 + (E.dZ[p] + 1) * 3 + (i0 - i) + 1];
    xb[(size_t)i * q + E.rt[p]] = cmk(c.x * E.sgn[p], c.y * E.sgn[p]);
  }
}

// Columns j0 .. j0 + B - 1 of a map: M[k][j0 + b] = x_b[k mod n][row(k / n)].
template <typename M>
__global__ void k_extract_map(const cplx* __restrict__ x, int n, int q, int r0, int r1, M* __restrict__ map,
                              int j0, int B) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (size_t)B * 2 * n) return;
  const int b = (int)(t % B), k = (int)(t / B);  // consecutive threads: one map row
  const int p = k / n, i = k % n;
  const cplx v = x[(size_t)b * n * q + (size_t)i * q + (p ? r1 : r0)];
  map[(size_t)k * 2 * n + j0 + b] = tmk<M>(v.x, v.y);
}

// Trace products of the decoupled sweep for a set of layers (blockIdx.y
// picks the layer), k < 2n:
//   out[k] = base[k] + sum_j M[k][j] x[j]            (base set)
//   out[k] = y[k mod n][row(k / n)] (+ x[k - n] for k >= n when addJ)
//            + sum_j M[k][j] x[j]                     (base null)
// with row(0) = r0, row(1) = r1, M [2n][2n] row-major or null.  WPR waves per
// output entry, eight loads of M and eight of x in flight per lane.  out
// may be base (each entry is read and written by the same lane).
template <typename T>
struct TraceSet {
  T* out[kSet];
  const T* base[kSet];
  const T* y[kSet];
  const T* M[kSet];
  const T* x[kSet];
  int q[kSet], r0[kSet], r1[kSet];
};

template <typename T, int WPR>
__global__ __launch_bounds__(256) void k_trace_set(TraceSet<T> S, int n, int addJ) {
  // WPR waves per output entry (4 / WPR entries per workgroup): wave part w
  // takes columns [w N2 / WPR, (w + 1) N2 / WPR) and the partial sums meet
  // in LDS
  __shared__ T red[4];
  const int z = blockIdx.y, w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int k = blockIdx.x * (4 / WPR) + w / WPR, part = w % WPR, N2 = 2 * n;
  if (k >= N2) return;  // with WPR = 4 the whole workgroup (k is uniform)
  const T* __restrict__ M = S.M[z];
  const T* __restrict__ x = S.x[z];
  T a0 = tmk<T>(0, 0), a1 = tmk<T>(0, 0);
  if (M) {
    const int j1 = part == WPR - 1 ? N2 : (part + 1) * (N2 / WPR);
    const T* row = M + (size_t)k * N2;
    int j = part * (N2 / WPR) + lane;
    for (; j + 7 * 64 < j1; j += 8 * 64) {
      T mv[8], xv[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        mv[u] = row[j + 64 * u];
        xv[u] = x[j + 64 * u];
      }
#pragma unroll
      for (int u = 0; u < 8; u += 2) {
        a0 = tfma(mv[u], xv[u], a0);
        a1 = tfma(mv[u + 1], xv[u + 1], a1);
      }
    }
    for (; j < j1; j += 64) a0 = tfma(row[j], x[j], a0);
  }
  T acc = tadd(a0, a1);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    acc.x += __shfl_xor(acc.x, off);
    acc.y += __shfl_xor(acc.y, off);
  }
  if constexpr (WPR > 1) {
    if (lane == 0) red[w] = acc;
    __syncthreads();
    if (w != 0) return;
#pragma unroll
    for (int u = 1; u < WPR; ++u) acc = tadd(acc, red[u]);
  }
  if (lane == 0) {
    T v;
    if (S.base[z]) {
      v = S.base[z][k];
    } else {
      v = S.y[z][(size_t)(k % n) * S.q[z] + (k < n ? S.r0[z] : S.r1[z])];
      if (addJ && k >= n) v = tadd(v, x[k - n]);
    }
    S.out[z][k] = tadd(v, acc);
  }
}

// Horizontal slabs (grid rows are the slab's short axis), many right-hand
// sides, no trace sources: the same copies as k_gather / k_scatter through
// a 64 (i) x 32 (r) LDS tile, so that both the grid rows (i fastest) and the
// slab rows (r fastest) are read and written in runs.
constexpr int kTI = 64, kTR = 32;
template <typename T>
__global__ __launch_bounds__(256) void k_gather_h(const T* __restrict__ g, T* __restrict__ dst, int n, int q,
                                                  int z0, int a, int b, T* __restrict__ dst2) {
  __shared__ T tile[kTR][kTI + 1];
  const int i0 = blockIdx.x * kTI, r0 = blockIdx.y * kTR;
  g += (size_t)blockIdx.z * n * n;
  dst += (size_t)blockIdx.z * n * q;
  const int tid = threadIdx.x;
#pragma unroll
  for (int e = 0; e < kTI * kTR / 256; ++e) {  // grid row Z = z0 + r, i fastest
    const int ii = tid % kTI, rr = tid / kTI + e * (256 / kTI);
    const int i = i0 + ii, Z = z0 + r0 + rr;
    tile[rr][ii] = (i < n && r0 + rr < q && Z >= a && Z <= b) ? g[(size_t)Z * n + i] : tmk<T>(0, 0);
  }
  __syncthreads();
#pragma unroll
  for (int e = 0; e < kTI * kTR / 256; ++e) {  // slab row i, r fastest
    const int rr = tid % kTR, ii = tid / kTR + e * (256 / kTR);
    const int i = i0 + ii, r = r0 + rr;
    if (i < n && r < q) {
      dst[(size_t)i * q + r] = tile[rr][ii];
      if (dst2) dst2[(size_t)blockIdx.z * n * q + (size_t)i * q + r] = tile[rr][ii];
    }
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_scatter_h(const T* __restrict__ src, T* __restrict__ out, int n, int q,
                                                   int z0, int a, int b, int accumulate) {
  __shared__ T tile[kTR][kTI + 1];
  const int i0 = blockIdx.x * kTI, Z0 = a + blockIdx.y * kTR;
  src += (size_t)blockIdx.z * n * q;
  out += (size_t)blockIdx.z * n * n;
  const int tid = threadIdx.x;
#pragma unroll
  for (int e = 0; e < kTI * kTR / 256; ++e) {  // slab row i, Z fastest
    const int rr = tid % kTR, ii = tid / kTR + e * (256 / kTR);
    const int i = i0 + ii, Z = Z0 + rr;
    if (i < n && Z <= b) tile[rr][ii] = src[(size_t)i * q + (Z - z0)];
  }
  __syncthreads();
#pragma unroll
  for (int e = 0; e < kTI * kTR / 256; ++e) {  // grid row Z, i fastest
    const int ii = tid % kTI, rr = tid / kTI + e * (256 / kTI);
    const int i = i0 + ii, Z = Z0 + rr;
    if (i < n && Z <= b) {
      const size_t o = (size_t)Z * n + i;
      out[o] = accumulate ? tadd(out[o], tile[rr][ii]) : tile[rr][ii];
    }
  }
}

// The same copies for one right-hand side, through narrower 16 (i) x 32 (r)
// tiles (enough workgroups for a single grid vector), with the trace
// sources folded in: the gather adds the downward sweep's sources to its
// tile before writing it out; the scatter's first row of tiles adds the
// upward sweep's sources of the next layer to that layer's right-hand side.
constexpr int kTI1 = 16;
template <typename T>
__global__ __launch_bounds__(128) void k_gather_h1(const T* __restrict__ g, T* __restrict__ dst, int n, int q,
                                                   int z0, int a, int b, const T* __restrict__ coef, Inject A,
                                                   Inject Bj, const T* __restrict__ sA) {
  __shared__ T tile[kTR][kTI1 + 1];
  const int i0 = blockIdx.x * kTI1, r0 = blockIdx.y * kTR;
  const int tid = threadIdx.x;
  // trace sources of this tile's columns: thread j < 16 line A, 16 <= j < 32 line B
  T inj = tmk<T>(0, 0);
  int injr = -1;
  if (sA && tid < 2 * kTI1) {
    const Inject& J = tid < kTI1 ? A : Bj;
    const int ii = tid % kTI1, i = i0 + ii;
    if (i < n && J.rt >= r0 && J.rt < r0 + kTR && J.rt < q) {
      inj = inject_term(coef, n, q, i, J, sA, (const T*)nullptr, 0, 0);
      injr = J.rt - r0;
    }
  }
#pragma unroll
  for (int e = 0; e < kTI1 * kTR / 128; ++e) {  // grid row Z = z0 + r, i fastest
    const int ii = tid % kTI1, rr = tid / kTI1 + e * (128 / kTI1);
    const int i = i0 + ii, Z = z0 + r0 + rr;
    tile[rr][ii] = (i < n && r0 + rr < q && Z >= a && Z <= b) ? g[(size_t)Z * n + i] : tmk<T>(0, 0);
  }
  __syncthreads();
  if (injr >= 0) tile[injr][tid % kTI1] = tadd(tile[injr][tid % kTI1], inj);
  __syncthreads();
#pragma unroll
  for (int e = 0; e < kTI1 * kTR / 128; ++e) {  // slab row i, r fastest
    const int rr = tid % kTR, ii = tid / kTR + e * (128 / kTR);
    const int i = i0 + ii, r = r0 + rr;
    if (i < n && r < q) dst[(size_t)i * q + r] = tile[rr][ii];
  }
}

template <typename T>
__global__ __launch_bounds__(128) void k_scatter_h1(const T* __restrict__ src, T* __restrict__ out, int n, int q,
                                                    int z0, int a, int b, int accumulate, T* __restrict__ rhs,
                                                    int qr, const T* __restrict__ coef, Inject A, Inject Bj,
                                                    const T* __restrict__ s2, int q2, int r2) {
  __shared__ T tile[kTR][kTI1 + 1];
  const int i0 = blockIdx.x * kTI1, Z0 = a + blockIdx.y * kTR;
  const int tid = threadIdx.x;
  const int t = i0 + tid;
  const bool inj = rhs && blockIdx.y == 0 && tid < kTI1 && t < n;
  T ta = tmk<T>(0, 0), tb = tmk<T>(0, 0), va = tmk<T>(0, 0), vb = tmk<T>(0, 0);
  if (inj) {  // the next layer's two trace sources, loads issued with the tile's
    ta = inject_term(coef, n, qr, t, A, src, (const T*)nullptr, 0, 0);
    tb = inject_term(coef, n, qr, t, Bj, src, s2, q2, r2);
    va = rhs[(size_t)t * qr + A.rt];
    vb = rhs[(size_t)t * qr + Bj.rt];
  }
#pragma unroll
  for (int e = 0; e < kTI1 * kTR / 128; ++e) {  // slab row i, Z fastest
    const int rr = tid % kTR, ii = tid / kTR + e * (128 / kTR);
    const int i = i0 + ii, Z = Z0 + rr;
    if (i < n && Z <= b) tile[rr][ii] = src[(size_t)i * q + (Z - z0)];
  }
  __syncthreads();
#pragma unroll
  for (int e = 0; e < kTI1 * kTR / 128; ++e) {  // grid row Z, i fastest
    const int ii = tid % kTI1, rr = tid / kTI1 + e * (128 / kTI1);
    const int i = i0 + ii, Z = Z0 + rr;
    if (i < n && Z <= b) {
      const size_t o = (size_t)Z * n + i;
      out[o] = accumulate ? tadd(out[o], tile[rr][ii]) : tile[rr][ii];
    }
  }
  if (inj) {
    rhs[(size_t)t * qr + A.rt] = tadd(va, ta);
    rhs[(size_t)t * qr + Bj.rt] = tadd(vb, tb);
  }
}

// Per-layer arguments of the decoupled sweep's multi-layer launches
// (blockIdx.z picks the layer): the layer's slab vector x (right-hand side
// or solution, [n][q]), its matrix, frame, and the two trace injections
// with their traces (null where the layer has no neighbour).
template <typename T>
struct LayerSet {
  T* x[kSet];
  const T* coef[kSet];
  int q[kSet], z0[kSet], a[kSet], b[kSet];
  TraceInj dn[kSet], up[kSet];
  const T* tau[kSet];
  const T* sig[kSet];
};

// x^l[i][r] = g(i, z0 + r) on the layer lines [a, b], 0 elsewhere, for
// every layer of the set; horizontal slabs through 16 (i) x 32 (r) LDS
// tiles as k_gather_h1 (grid rows read and slab rows written in runs).
template <typename T>
__global__ __launch_bounds__(128) void k_gather_set_h(const T* __restrict__ g, LayerSet<T> S, int n) {
  __shared__ T tile[kTR][16 + 1];
  const int z = blockIdx.z, q = S.q[z], z0 = S.z0[z], a = S.a[z], b = S.b[z];
  const int i0 = blockIdx.x * 16, r0 = blockIdx.y * kTR;
  if (r0 >= q) return;  // whole workgroup, before any barrier
  T* __restrict__ dst = S.x[z];
  const int tid = threadIdx.x;
#pragma unroll
  for (int e = 0; e < 16 * kTR / 128; ++e) {  // grid row Z = z0 + r, i fastest
    const int ii = tid % 16, rr = tid / 16 + e * (128 / 16);
    const int i = i0 + ii, Z = z0 + r0 + rr;
    tile[rr][ii] = (i < n && r0 + rr < q && Z >= a && Z <= b) ? g[(size_t)Z * n + i] : tmk<T>(0, 0);
  }
  __syncthreads();
#pragma unroll
  for (int e = 0; e < 16 * kTR / 128; ++e) {  // slab row i, r fastest
    const int rr = tid % kTR, ii = tid / kTR + e * (128 / kTR);
    const int i = i0 + ii, r = r0 + rr;
    if (i < n && r < q) dst[(size_t)i * q + r] = tile[rr][ii];
  }
}

// The same for vertical slabs (the short axis is the grid's fast axis).
template <typename T>
__global__ void k_gather_set_v(const T* __restrict__ g, LayerSet<T> S, int n) {
  const int z = blockIdx.z, q = S.q[z];
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (size_t)n * q) return;
  const int i = (int)(t / q), r = (int)(t % q), Z = S.z0[z] + r;
  S.x[z][t] = (Z >= S.a[z] && Z <= S.b[z]) ? g[(size_t)i * n + Z] : tmk<T>(0, 0);
}

// x^l += E^l tau^{l+1} + F^l sigma^{l-1} for every layer of the set: line
// part p of a trace enters row rt[p] of the layer through the stencil
// couplings of row dZ[p], times sgn[p] (a null trace adds nothing).
template <typename T>
__global__ void k_inject_set(LayerSet<T> S, int n) {
  const int z = blockIdx.z, i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int q = S.q[z];
  const T* __restrict__ coef = S.coef[z];
  T* __restrict__ rhs = S.x[z];
  for (int s = 0; s < 2; ++s) {
    const TraceInj& J = s ? S.up[z] : S.dn[z];
    const T* tr = s ? S.sig[z] : S.tau[z];
    if (!tr) continue;
    for (int p = 0; p < 2; ++p) {
      const T* cf = coef + ((size_t)i * q + J.rt[p]) * 9 + (J.dZ[p] + 1) * 3;
      T acc = tmk<T>(0, 0);
      for (int dX = -1; dX <= 1; ++dX) {
        const int ii = i + dX;
        if (ii < 0 || ii >= n) continue;
        acc = tfma(cf[dX + 1], tr[(size_t)p * n + ii], acc);
      }
      T* o = rhs + (size_t)i * q + J.rt[p];
      *o = tadd(*o, tmk<T>(acc.x * J.sgn[p], acc.y * J.sgn[p]));
    }
  }
}

// out(i, Z) (+)= x^l[i][Z - z0] for the layer lines Z in [a, b] of every
// layer of the set (disjoint rows of out); horizontal slabs through LDS
// tiles as k_scatter_h1.
template <typename T>
__global__ __launch_bounds__(128) void k_scatter_set_h(T* __restrict__ out, LayerSet<T> S, int n, int accumulate) {
  __shared__ T tile[kTR][16 + 1];
  const int z = blockIdx.z, q = S.q[z], z0 = S.z0[z], a = S.a[z], b = S.b[z];
  const int i0 = blockIdx.x * 16, Z0 = a + blockIdx.y * kTR;
  if (Z0 > b) return;  // whole workgroup, before any barrier
  const T* __restrict__ src = S.x[z];
  const int tid = threadIdx.x;
#pragma unroll
  for (int e = 0; e < 16 * kTR / 128; ++e) {  // slab row i, Z fastest
    const int rr = tid % kTR, ii = tid / kTR + e * (128 / kTR);
    const int i = i0 + ii, Z = Z0 + rr;
    if (i < n && Z <= b) tile[rr][ii] = src[(size_t)i * q + (Z - z0)];
  }
  __syncthreads();
#pragma unroll
  for (int e = 0; e < 16 * kTR / 128; ++e) {  // grid row Z, i fastest
    const int ii = tid % 16, rr = tid / 16 + e * (128 / 16);
    const int i = i0 + ii, Z = Z0 + rr;
    if (i < n && Z <= b) {
      const size_t o = (size_t)Z * n + i;
      out[o] = accumulate ? tadd(out[o], tile[rr][ii]) : tile[rr][ii];
    }
  }
}

template <typename T>
__global__ void k_scatter_set_v(T* __restrict__ out, LayerSet<T> S, int n, int accumulate) {
  const int z = blockIdx.z, a = S.a[z], rows = S.b[z] - a + 1;
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (size_t)n * rows) return;
  const int i = (int)(t / rows), Z = a + (int)(t % rows);
  const T v = S.x[z][(size_t)i * S.q[z] + (Z - S.z0[z])];
  const size_t o = (size_t)i * n + Z;
  out[o] = accumulate ? tadd(out[o], v) : v;
}

__global__ void k_down_copy(const cplx* __restrict__ a, fcplx* __restrict__ b, size_t cnt) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < cnt) b[i] = make_float2((float)a[i].x, (float)a[i].y);
}

template <typename K>
hipError_t set_lds(K kernel, size_t bytes) {
  if (bytes <= 65536) return hipSuccess;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

// Launch of one batched level step: the widest tile shape that still gives
// at least two workgroups per CU, never wider than the batch needs.
template <typename C, int MODE, int V>
static void bstep_go(ls_plan* p, C* x, size_t xs_b, int B, const C* a0, const C* a1, const C* a2,
                     const C* coef, int q, int nl, int shift, int nb) {
  constexpr int BT = BVariants<C>::BT[V], NT = BVariants<C>::NT[V];
  const int tiles = (B + BT - 1) / BT;
  const int total = nb * tiles;
  k_bstep<C, MODE, BT, NT><<<total, NT, BShape<C, BT, NT>::lds(), p->stream>>>(
      x, xs_b, B, a0, a1, a2, coef, p->n, q, nl, shift, tiles, total);
}

template <typename C, int MODE>
static void bstep(ls_plan* p, C* x, size_t xs_b, int B, const C* a0, const C* a1, const C* a2,
                  const C* coef, int q, int nl, int shift, int nb) {
  if constexpr (std::is_same<C, fcplx>::value) {
    // matrix cores when the level has enough (block, 32-RHS tile) pairs
    const int tiles = (B + kMB - 1) / kMB;
    // (block, tile) pairs >= 256 measured best against 64 and 128 thresholds
    if (B >= 16 && (long)nb * tiles >= 256) {
      static const hipError_t once = set_lds(k_bstep_mfma<MODE>, bstep_mfma_lds<MODE>(kMaxQ));
      (void)once;
      const int total = nb * tiles;
      k_bstep_mfma<MODE><<<total, 64 * ((q + 15) / 16), bstep_mfma_lds<MODE>(q), p->stream>>>(
          x, xs_b, B, a0, a1, a2, coef, p->n, q, nl, shift, tiles, total);
      return;
    }
  }
  using V = BVariants<C>;
  int v = 2;
  for (int i = 0; i < 2; ++i) {
    if (V::BT[i + 1] >= B) continue;  // a narrower tile already holds the batch
    if ((long)nb * ((B + V::BT[i] - 1) / V::BT[i]) >= 512) { v = i; break; }
    v = i + 1;
  }
  if (v == 0)
    bstep_go<C, MODE, 0>(p, x, xs_b, B, a0, a1, a2, coef, q, nl, shift, nb);
  else if (v == 1)
    bstep_go<C, MODE, 1>(p, x, xs_b, B, a0, a1, a2, coef, q, nl, shift, nb);
  else
    bstep_go<C, MODE, 2>(p, x, xs_b, B, a0, a1, a2, coef, q, nl, shift, nb);
}

// Top operator of one slab from its FP64 factors: the levels from the
// first with at most kTopBlocks blocks up to the top and back, applied to the
// Nt identity columns in a compact frame [Nt][nl][q] (row j of that level at
// j; level l >= top_level then has shift l - top_level), then transposed to
// row-major.  work: work_cap complex scratch; a slab whose Nt^2 does not fit
// keeps the level-by-level chain.
static ls_status build_top(ls_plan* p, Slab& s, const cplx* fac, cplx* work, size_t work_cap) {
  const int nlev = (int)s.levels.size();
  const int lim = (p->opt.sweep == LS_SWEEP_DECOUPLED && p->opt.max_batch < kTopBatchMin) ? kTopBlocksDec
                                                                                          : kTopBlocks;
  int ls = -1;
  for (int l = 1; l < nlev; ++l)
    if (s.levels[l].nl <= lim) {
      ls = l;
      break;
    }
  s.top_level = -1;
  s.top_n = 0;
  if (ls < 1 || s.levels[ls].nl < 2) return LS_OK;
  const int q = s.q, Nt = s.levels[ls].nl * q;
  if ((size_t)Nt * Nt > work_cap || Nt > kTopMax) return LS_OK;
  const int blocks = (int)std::min<size_t>(4096, ((size_t)Nt * Nt + 255) / 256);
  k_identity<<<blocks, 256, 0, p->stream>>>(work, Nt);
  for (int l = ls; l < nlev - 1; ++l) {
    const SlabLevel& L = s.levels[l];
    bstep<cplx, BSTEP_FWD>(p, work, (size_t)Nt, Nt, fac + L.off_pm, fac + L.off_pp, nullptr, s.coef, q,
                           L.nl, l - ls, (L.nl + 1) / 2);
  }
  bstep<cplx, BSTEP_LAST>(p, work, (size_t)Nt, Nt, fac + s.levels[nlev - 1].off_dinv, nullptr, nullptr,
                          s.coef, q, 1, 0, 1);
  for (int l = nlev - 2; l >= ls; --l) {
    const SlabLevel& L = s.levels[l];
    bstep<cplx, BSTEP_BWD>(p, work, (size_t)Nt, Nt, fac + L.off_dinv, fac + L.off_dinvl, fac + L.off_dinvu,
                           s.coef, q, L.nl, l - ls, L.nl / 2);
  }
  const size_t bytes = (size_t)Nt * Nt;
  if (p->fp32) {
    LS_TRY(plan_alloc(p, (void**)&s.top32, bytes * sizeof(fcplx)));
    k_transpose_to<fcplx><<<blocks, 256, 0, p->stream>>>(work, s.top32, Nt);
    if (p->opt.max_batch >= kTopBatchMin) {  // column-major copy for many right-hand sides
      LS_TRY(plan_alloc(p, (void**)&s.top32T, bytes * sizeof(fcplx)));
      k_down_copy<<<(unsigned)((bytes + 255) / 256), 256, 0, p->stream>>>(work, s.top32T, bytes);
      if (!p->top_part32)
        LS_TRY(plan_alloc(p, (void**)&p->top_part32,
                          (size_t)kTopSlices * kTopMax * p->opt.max_batch * sizeof(fcplx)));
    }
  } else {
    LS_TRY(plan_alloc(p, (void**)&s.top, bytes * sizeof(cplx)));
    k_transpose_to<cplx><<<blocks, 256, 0, p->stream>>>(work, s.top, Nt);
  }
  LS_HIP(hipGetLastError());
  s.top_level = ls;
  s.top_n = Nt;
  return LS_OK;
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

template <typename C>
static ls_status solve_levels_b(ls_plan* p, const Slab& s, const C* fac, const C* coef, C* x, size_t xs_b, int B);

// Trace sources of layer s: from the layer above (downward sweep: lines b + 1
// and b of its solution, into rows b and b + 1) and from the layer below
// (upward sweep: lines a - 1 and a, into rows a and a - 1).
static TraceInj inj_down(const Slab& s) {
  return TraceInj{{s.b - s.z0, s.b + 1 - s.z0}, {+1, -1}, {-1.0, +1.0}};
}
static TraceInj inj_up(const Slab& s) {
  return TraceInj{{s.a - s.z0, s.a - 1 - s.z0}, {-1, +1}, {-1.0, +1.0}};
}

// Trace-transfer maps of layer s (decoupled sweep), from its FP64 factors:
// (C^l)^{-1} applied to the 2n unit traces of each injection it needs (in
// batches of solves on `work`), restricted to the two lines each neighbour
// reads.  Layer l of L needs mT (1 <= l <= L-2), mU (l <= L-2), mV
// (1 <= l <= L-2).
static ls_status build_maps(ls_plan* p, Slab& s, const cplx* fac, cplx* work, size_t work_elems) {
  const int n = p->n, q = s.q, l = s.idx, L = p->L, N2 = 2 * n;
  const bool needT = l >= 1 && l <= L - 2, needU = l <= L - 2, needV = l >= 1 && l <= L - 2;
  if (!needU) return LS_OK;
  const size_t mbytes = (size_t)N2 * N2 * (p->fp32 ? sizeof(fcplx) : sizeof(cplx));
  void* mT = nullptr;
  void* mU = nullptr;
  void* mV = nullptr;
  if (needT) LS_TRY(plan_alloc(p, &mT, mbytes));
  LS_TRY(plan_alloc(p, &mU, mbytes));
  if (needV) LS_TRY(plan_alloc(p, &mV, mbytes));
  const size_t vec = (size_t)n * q;
  const int Bc = (int)std::max<size_t>(1, std::min<size_t>(256, work_elems / vec));
  const int rows_tau[2] = {s.a - s.z0, s.a - 1 - s.z0};
  const int rows_sig[2] = {s.b - s.z0, s.b + 1 - s.z0};
  auto extract = [&](void* map, const int* rows, int j0, int B) -> ls_status {
    const size_t cnt = (size_t)B * N2;
    const unsigned blocks = (unsigned)((cnt + 255) / 256);
    if (p->fp32)
      k_extract_map<fcplx><<<blocks, 256, 0, p->stream>>>(work, n, q, rows[0], rows[1], (fcplx*)map, j0, B);
    else
      k_extract_map<cplx><<<blocks, 256, 0, p->stream>>>(work, n, q, rows[0], rows[1], (cplx*)map, j0, B);
    LS_HIP(hipGetLastError());
    return LS_OK;
  };
  for (int which = 0; which < 2; ++which) {  // 0: downward injection E, 1: upward F
    if (which == 1 && !needV) break;
    const TraceInj J = which == 0 ? inj_down(s) : inj_up(s);
    for (int j0 = 0; j0 < N2; j0 += Bc) {
      const int B = std::min(Bc, N2 - j0);
      LS_HIP(hipMemsetAsync(work, 0, (size_t)B * vec * sizeof(cplx), p->stream));
      k_unit_rhs<<<(B + 63) / 64, 64, 0, p->stream>>>(work, s.coef, n, q, J, j0, B);
      LS_HIP(hipGetLastError());
      LS_TRY(solve_levels_b<cplx>(p, s, fac, s.coef, work, vec, B));
      if (which == 0) {
        if (needT) LS_TRY(extract(mT, rows_tau, j0, B));
        LS_TRY(extract(mU, rows_sig, j0, B));
      } else {
        LS_TRY(extract(mV, rows_sig, j0, B));
      }
    }
  }
  LS_HIP(hipStreamSynchronize(p->stream));
  if (p->fp32) {
    s.mT32 = (fcplx*)mT;
    s.mU32 = (fcplx*)mU;
    s.mV32 = (fcplx*)mV;
  } else {
    s.mT = (cplx*)mT;
    s.mU = (cplx*)mU;
    s.mV = (cplx*)mV;
  }
  return LS_OK;
}

// Layers (Section 3.1): t = n / L lines each, the first n mod L layers one
// more; extension ext lines each side, clipped to the grid.
// Two slabs can share multi-slab launches: same thickness, the same levels
// (block counts and factor offsets) and the same top operator shape.
static bool same_shape(const Slab& x, const Slab& y) {
  if (x.q != y.q || x.levels.size() != y.levels.size() || x.top_level != y.top_level || x.top_n != y.top_n ||
      x.fac_elems != y.fac_elems)
    return false;
  for (size_t l = 0; l < x.levels.size(); ++l) {
    const SlabLevel &a = x.levels[l], &b = y.levels[l];
    if (a.nl != b.nl || a.off_dinv != b.off_dinv || a.off_dinvl != b.off_dinvl || a.off_dinvu != b.off_dinvu ||
        a.off_pm != b.off_pm || a.off_pp != b.off_pp)
      return false;
  }
  return true;
}

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
  cplx* fac64 = nullptr;  // FP32 plans: FP64 factors of one slab before rounding
  int* status = nullptr;
  LS_HIP(hipMalloc(&work, work_elems * sizeof(cplx)));
  if (p->fp32) {
    size_t mx = 0;
    for (int o = 0; o < 2; ++o)
      for (Slab& s : p->slabs[o]) mx = std::max(mx, plan_levels(s, n));
    LS_HIP(hipMalloc(&fac64, mx * sizeof(cplx)));
  }
  LS_HIP(hipMalloc(&status, sizeof(int)));
  LS_HIP(hipMemsetAsync(status, 0, sizeof(int), p->stream));
  unsigned* tri_worst = nullptr;  // largest elimination-vs-inverse difference (float bits)
  LS_HIP(hipMalloc(&tri_worst, sizeof(unsigned)));
  LS_HIP(hipMemsetAsync(tri_worst, 0, sizeof(unsigned), p->stream));
  bool tri_all = true;            // every slab has level-0 odd blocks to factor
  const double w2 = p->omega * p->omega;
  const double sigma = p->opt.shift_c / p->omega;
  ls_status st = LS_OK;
  for (int o = 0; o < 2 && st == LS_OK; ++o) {
    for (Slab& s : p->slabs[o]) {
      const size_t cbytes = (size_t)n * s.q * 9 * sizeof(cplx);
      const size_t vec = (size_t)n * s.q;
      const size_t bvec = vec * p->opt.max_batch;
      if ((st = plan_alloc(p, (void**)&s.coef, cbytes)) != LS_OK) break;
      s.fac_elems = plan_levels(s, n);
      if (p->fp32) {
        if ((st = plan_alloc(p, (void**)&s.coef32, cbytes / 2)) != LS_OK) break;
        if ((st = plan_alloc(p, (void**)&s.g32, bvec * sizeof(fcplx))) != LS_OK) break;
        if ((st = plan_alloc(p, (void**)&s.w32, bvec * sizeof(fcplx))) != LS_OK) break;
        if ((st = plan_alloc(p, (void**)&s.fac32, s.fac_elems * sizeof(fcplx))) != LS_OK) break;
        s.fac = fac64;
      } else {
        if ((st = plan_alloc(p, (void**)&s.g, bvec * sizeof(cplx))) != LS_OK) break;
        if ((st = plan_alloc(p, (void**)&s.w, bvec * sizeof(cplx))) != LS_OK) break;
        if ((st = plan_alloc(p, (void**)&s.fac, s.fac_elems * sizeof(cplx))) != LS_OK) break;
      }
      const cplx* tables = p->stencil_d + (o == 0 ? 0 : 162);
      const double t0 = plan_clock_ms(p);
      k_assemble<<<dim3((s.q + 63) / 64, n), 64, 0, p->stream>>>(
          s.coef, tables, p->m, n, s.q, s.z0, s.a, s.b, std::max(ext, 2), o, w2, sigma);
      if (hipGetLastError() != hipSuccess) { ls_set_error("assembly launch failed"); st = LS_EDEVICE; break; }
      {  // level-0 coupling table in the plan's precision
        const size_t ce = (size_t)n * 6 * s.q;
        const unsigned cb = (unsigned)((ce + 255) / 256);
        if (p->fp32) {
          if ((st = plan_alloc(p, (void**)&s.cpl32, ce * sizeof(fcplx))) != LS_OK) break;
          k_couplings<fcplx><<<cb, 256, 0, p->stream>>>(s.coef, s.cpl32, n, s.q);
        } else {
          if ((st = plan_alloc(p, (void**)&s.cpl, ce * sizeof(cplx))) != LS_OK) break;
          k_couplings<cplx><<<cb, 256, 0, p->stream>>>(s.coef, s.cpl, n, s.q);
        }
        if (hipGetLastError() != hipSuccess) { ls_set_error("coupling table launch failed"); st = LS_EDEVICE; break; }
      }
      const double t1 = plan_clock_ms(p);
      if ((st = factor_slab(p, s, work, status)) != LS_OK) break;
      const double t2 = plan_clock_ms(p);
      if ((st = build_top(p, s, s.fac, work, work_elems)) != LS_OK) break;
      const double t3 = plan_clock_ms(p);
      if (p->opt.sweep == LS_SWEEP_DECOUPLED && (st = build_maps(p, s, s.fac, work, work_elems)) != LS_OK) break;
      const double t4 = plan_clock_ms(p);
      if (s.levels.size() > 1 && n >= 2) {
        // level-0 odd blocks' tridiagonal factors, each block's elimination
        // checked against its dense inverse (FP64 factors for the check)
        const int no = n / 2;
        const size_t te = (size_t)3 * s.q * no;
        const unsigned tb = (unsigned)(((size_t)no * s.q + 255) / 256);
        cplx* t64 = work;
        if (!p->fp32) {
          if ((st = plan_alloc(p, (void**)&s.tri, te * sizeof(cplx))) != LS_OK) break;
          t64 = s.tri;
        }
        k_tri_coef<cplx><<<tb, 256, 0, p->stream>>>(s.coef, t64, n, s.q);
        if (s.q <= kPcrRows)
          k_tri_check<<<no, 64, 0, p->stream>>>(t64, s.fac + s.levels[0].off_dinv, n, s.q, tri_worst);
        else
          tri_all = false;
        if (p->fp32) {
          if ((st = plan_alloc(p, (void**)&s.tri32, te * sizeof(fcplx))) != LS_OK) break;
          k_tri_coef<fcplx><<<tb, 256, 0, p->stream>>>(s.coef, s.tri32, n, s.q);
        }
        if (hipGetLastError() != hipSuccess) { ls_set_error("tridiagonal factor launch failed"); st = LS_EDEVICE; break; }
      } else {
        tri_all = false;
      }
      p->stage_ms[4] += plan_clock_ms(p) - t4;
      p->stage_ms[3] += t1 - t0;
      p->stage_ms[4] += t2 - t1;
      p->stage_ms[5] += t3 - t2;
      p->stage_ms[6] += t4 - t3;
      if (p->fp32) {
        // FP64 factorisation, FP32 storage for the solves
        k_down_copy<<<(unsigned)((s.fac_elems + 255) / 256), 256, 0, p->stream>>>(s.fac, s.fac32,
                                                                              s.fac_elems);
        k_down_copy<<<(unsigned)((vec * 9 + 255) / 256), 256, 0, p->stream>>>(s.coef, s.coef32,
                                                                            vec * 9);
        if (hipGetLastError() != hipSuccess || hipStreamSynchronize(p->stream) != hipSuccess) {
          ls_set_error("factor conversion failed");
          st = LS_EDEVICE;
          break;
        }
        s.fac = nullptr;
      }
    }
  }
  int bad = 0;
  unsigned worst_bits = 0;
  if (st == LS_OK) {
    if (hipMemcpy(&bad, status, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(&worst_bits, tri_worst, sizeof(unsigned), hipMemcpyDeviceToHost) != hipSuccess)
      st = LS_EDEVICE;
  }
  (void)hipFree(work);
  if (fac64) (void)hipFree(fac64);
  (void)hipFree(status);
  (void)hipFree(tri_worst);
  {
    float worst;
    std::memcpy(&worst, &worst_bits, sizeof(worst));
    p->tri_ok = p->opt.level0 == LS_LEVEL0_AUTO && tri_all && worst <= 1e-9f;
  }
  if (st != LS_OK) return st;
  if (bad) {
    ls_set_error("slab factorisation: zero or non-finite pivot");
    return LS_ESINGULAR;
  }
  if (p->opt.sweep == LS_SWEEP_DECOUPLED) {
    const size_t tr = (size_t)2 * L * 2 * n;
    if (p->fp32) LS_TRY(plan_alloc(p, (void**)&p->traces32, tr * sizeof(fcplx)));
    else LS_TRY(plan_alloc(p, (void**)&p->traces, tr * sizeof(cplx)));
    // layers grouped by slab shape (at most kSet per group), every layer's
    // elimination scratch, side streams (default priority) for the groups
    for (int o = 0; o < 2; ++o) {
      std::vector<std::vector<int>>& G = p->dec_groups[o];
      G.clear();
      const std::vector<Slab>& S = p->slabs[o];
      for (int l = 0; l < (int)S.size(); ++l) {
        bool placed = false;
        for (auto& grp : G)
          if ((int)grp.size() < kSet && same_shape(S[grp[0]], S[l])) {
            grp.push_back(l);
            placed = true;
            break;
          }
        if (!placed) G.push_back({l});
      }
      std::stable_sort(G.begin(), G.end(), [](const std::vector<int>& x, const std::vector<int>& y) {
        return x.size() > y.size();
      });
    }
    const size_t esz = p->fp32 ? sizeof(fcplx) : sizeof(cplx);
    const size_t Lmax = std::max(p->slabs[0].size(), p->slabs[1].size());
    p->set_qmax = qmax;
    LS_TRY(plan_alloc(p, &p->set_elim, Lmax * n * qmax * esz));
    LS_HIP(hipEventCreateWithFlags(&p->side_fork, hipEventDisableTiming));
    for (int k = 0; k < ls_plan::kSide; ++k) {
      LS_HIP(hipStreamCreateWithFlags(&p->side[k], hipStreamNonBlocking));
      LS_HIP(hipEventCreateWithFlags(&p->side_join[k], hipEventDisableTiming));
    }
  }
  const size_t wv = (size_t)n * qmax * p->opt.max_batch;
  const size_t w1 = (size_t)n * qmax;  // single-right-hand-side elimination scratch
  if (p->fp32) {
    LS_TRY(plan_alloc(p, (void**)&p->slab_work32, wv * sizeof(fcplx)));
    LS_TRY(plan_alloc(p, (void**)&p->slab_work32b, wv * sizeof(fcplx)));
    LS_TRY(plan_alloc(p, (void**)&p->slab_elim32, w1 * sizeof(fcplx)));
  } else {
    LS_TRY(plan_alloc(p, (void**)&p->slab_work, wv * sizeof(cplx)));
    LS_TRY(plan_alloc(p, (void**)&p->slab_work2, wv * sizeof(cplx)));
    LS_TRY(plan_alloc(p, (void**)&p->slab_elim, w1 * sizeof(cplx)));
  }
  return LS_OK;
}

template <typename C>
static ls_status solve_levels_b(ls_plan* p, const Slab& s, const C* fac, const C* coef, C* x,
                                size_t xs_b, int B) {
  const int n = p->n, q = s.q;
  const int nlev = (int)s.levels.size();
  if (nlev == 1) {
    bstep<C, BSTEP_LAST>(p, x, xs_b, B, fac + s.levels[0].off_dinv, nullptr, nullptr, coef, q, 1,
                         0, 1);
    LS_HIP(hipGetLastError());
    return LS_OK;
  }
  const SlabLevel& L0 = s.levels[0];
  // levels from the top level up as one dense operator (FP32, many right-hand sides)
  int top_l = nlev - 1;
  const fcplx* topT = nullptr;
  if constexpr (std::is_same<C, fcplx>::value) {
    if (B >= kTopBatchMin && s.top_level >= 1 && s.top32T && p->top_part32) {
      top_l = s.top_level;
      topT = s.top32T;
    }
  }
  bstep<C, BSTEP_ODD0>(p, x, xs_b, B, fac + L0.off_dinv, nullptr, nullptr, coef, q, L0.nl, 0,
                       L0.nl / 2);
  constexpr int RB = sizeof(C) == 8 ? 4 : 2;  // right-hand sides per thread (no spills)
  k_fwd0_even_b<C, RB><<<dim3((q + 127) / 128, (L0.nl + 1) / 2, (B + RB - 1) / RB), 128, 0, p->stream>>>(
      x, xs_b, coef, n, q, B);
  for (int l = 1; l < top_l; ++l) {
    const SlabLevel& L = s.levels[l];
    bstep<C, BSTEP_FWD>(p, x, xs_b, B, fac + L.off_pm, fac + L.off_pp, nullptr, coef, q, L.nl, l,
                        (L.nl + 1) / 2);
  }
  if constexpr (std::is_same<C, fcplx>::value) {
    if (topT) {
      const int Nt = s.top_n, slices = (Nt + kTopKL - 1) / kTopKL;
      k_top_mfma<<<dim3((Nt + 63) / 64, (B + kMB - 1) / kMB, slices), 256, 0, p->stream>>>(
          topT, x, xs_b, B, Nt, q, top_l, p->top_part32);
      k_top_reduce<<<(unsigned)(((size_t)Nt * B + 255) / 256), 256, 0, p->stream>>>(p->top_part32, slices, Nt, B,
                                                                                     x, xs_b, q, top_l);
    }
  }
  if (top_l == nlev - 1)
    bstep<C, BSTEP_LAST>(p, x, xs_b, B, fac + s.levels[nlev - 1].off_dinv, nullptr, nullptr, coef,
                         q, 1, 0, 1);
  for (int l = top_l - 1; l >= 1; --l) {
    const SlabLevel& L = s.levels[l];
    bstep<C, BSTEP_BWD>(p, x, xs_b, B, fac + L.off_dinv, fac + L.off_dinvl, fac + L.off_dinvu,
                        coef, q, L.nl, l, L.nl / 2);
  }
  bstep<C, BSTEP_BWD0>(p, x, xs_b, B, fac + L0.off_dinv, nullptr, nullptr, coef, q, L0.nl, 0,
                       L0.nl / 2);
  LS_HIP(hipGetLastError());
  return LS_OK;
}

// One right-hand side per slab: y = C_slab^{-1} g (g untouched, t scratch)
// for the cnt <= kSet slabs of S, which share s's q and level structure.
// Rows of the level-0 odd blocks to complete (the rest of those blocks
// keeps intermediate values): all, the lists S.sel, or the ranges
// [S.lo, S.hi).
enum { ROWS_ALL = 0, ROWS_SEL = 1, ROWS_RANGE = 2 };
template <typename C>
static ls_status solve_rows_set(ls_plan* p, const Slab& s, const SlabSet<C>& S, int cnt, int rows = ROWS_ALL) {
  const int n = p->n, q = s.q;
  const int nlev = (int)s.levels.size();
  auto step = [&](auto kern, auto mode, int nb, size_t o0, size_t o1, size_t o2, int nl, int shift) {
    using RC = RCols<decltype(mode)::value>;
    const int RS = row_splits(q, RC::T, RC::N);
    kern<<<dim3(nb * RS, cnt), 256, 0, p->stream>>>(S, o0, o1, o2, n, q, nl, shift, RS);
  };
  using ModeOdd0 = std::integral_constant<int, R_ODD0>;
  using ModeFwd = std::integral_constant<int, R_FWD>;
  using ModeLast = std::integral_constant<int, R_LAST>;
  using ModeBwd = std::integral_constant<int, R_BWD>;
  using ModeBwd0 = std::integral_constant<int, R_BWD0>;
  if (nlev == 1) {  // a single block row
    for (int z = 0; z < cnt; ++z)
      LS_HIP(hipMemcpyAsync(S.t[z], S.g[z], sizeof(C) * q, hipMemcpyDeviceToDevice, p->stream));
    step(k_rstep<C, R_LAST>, ModeLast{}, 1, s.levels[0].off_dinv, 0, 0, 1, 0);
    LS_HIP(hipGetLastError());
    return LS_OK;
  }
  const SlabLevel& L0 = s.levels[0];
  // level-0 odd blocks by the tridiagonal elimination where the plan keeps
  // its factors, else by their dense inverses
  const bool tri = S.tri[0] != nullptr;
  const dim3 tgrid(n / 2, cnt);
  if (tri)
    k_tri_odd0<C><<<tgrid, 64, 0, p->stream>>>(S, n, q);
  else
    step(k_rstep<C, R_ODD0>, ModeOdd0{}, L0.nl / 2, L0.off_dinv, 0, 0, L0.nl, 0);
  k_even0<C><<<dim3((((n + 1) / 2) * q + 255) / 256, cnt), 256, 0, p->stream>>>(S, n, q);
  // levels from `top` up: one dense operator when the plan built it
  const int top_l = (s.top_level >= 1 && S.top[0]) ? s.top_level : nlev - 1;
  // level 1 with its couplings through the tridiagonal level-0 blocks (only
  // D'^{-1} of its odd blocks read) when it is a level of its own and the
  // launch takes several slabs (for one slab its coupling waves, n/4, are
  // too few to hide their latency: the dense steps are faster there)
  const bool l1 = tri && top_l >= 2 && cnt >= 2;
  using ModeOddL = std::integral_constant<int, R_ODDL>;
  for (int l = 1; l < top_l; ++l) {
    const SlabLevel& L = s.levels[l];
    if (l == 1 && l1) {
      step(k_rstep<C, R_ODDL>, ModeOddL{}, L.nl / 2, L.off_dinv, 0, 0, L.nl, 1);
      k_l1_couple<C><<<dim3((L.nl + 1) / 2, cnt), 64, 0, p->stream>>>(S, n, q, 0);
    } else {
      step(k_rstep<C, R_FWD>, ModeFwd{}, (L.nl + 1) / 2, L.off_pm, L.off_pp, 0, L.nl, l);
    }
  }
  if (top_l < nlev - 1) {
    k_top<C><<<dim3((s.top_n + 3) / 4, cnt), 256, 0, p->stream>>>(S, s.top_n, q, top_l);
  } else {
    step(k_rstep<C, R_LAST>, ModeLast{}, 1, s.levels[nlev - 1].off_dinv, 0, 0, 1, 0);
  }
  for (int l = top_l - 1; l >= 1; --l) {
    const SlabLevel& L = s.levels[l];
    if (l == 1 && l1) {
      k_l1_couple<C><<<dim3(L.nl / 2, cnt), 64, 0, p->stream>>>(S, n, q, 2);
      step(k_rstep<C, R_ODDL>, ModeOddL{}, L.nl / 2, L.off_dinv, 0, 0, L.nl, 1);
    } else {
      step(k_rstep<C, R_BWD>, ModeBwd{}, L.nl / 2, L.off_dinv, L.off_dinvl, L.off_dinvu, L.nl, l);
    }
  }
  k_odd0_lu<C><<<dim3(((n / 2) * q + 255) / 256, cnt), 256, 0, p->stream>>>(S, n, q);
  if (tri) {
    if (rows == ROWS_SEL) k_tri_bwd0<C, ROWS_SEL><<<tgrid, 64, 0, p->stream>>>(S, n, q);
    else if (rows == ROWS_RANGE) k_tri_bwd0<C, ROWS_RANGE><<<tgrid, 64, 0, p->stream>>>(S, n, q);
    else k_tri_bwd0<C, ROWS_ALL><<<tgrid, 64, 0, p->stream>>>(S, n, q);
  } else if (rows == ROWS_SEL) {  // one tile of the selected rows per block
    k_rstep<C, R_BWD0S><<<dim3(L0.nl / 2, cnt), 256, 0, p->stream>>>(S, L0.off_dinv, 0, 0, n, q, L0.nl, 0, 1);
  } else if (rows == ROWS_RANGE) {  // tiles over the longest range of the set
    int span = 1;
    for (int z = 0; z < cnt; ++z) span = std::max(span, S.hi[z] - S.lo[z]);
    const int RS = row_splits(span, q, RCols<R_BWD0R>::T, RCols<R_BWD0R>::N);
    k_rstep<C, R_BWD0R><<<dim3(L0.nl / 2 * RS, cnt), 256, 0, p->stream>>>(S, L0.off_dinv, 0, 0, n, q, L0.nl, 0, RS);
  } else {
    step(k_rstep<C, R_BWD0>, ModeBwd0{}, L0.nl / 2, L0.off_dinv, 0, 0, L0.nl, 0);
  }
  LS_HIP(hipGetLastError());
  return LS_OK;
}

// One right-hand side of one slab.
template <typename C>
static ls_status solve_rows(ls_plan* p, const Slab& s, const C* fac, const C* coef, const C* cpl, const C* tri,
                            const C* top, const C* g, C* t, C* y) {
  SlabSet<C> S{};
  S.tri[0] = tri;
  S.g[0] = g;
  S.t[0] = t;
  S.y[0] = y;
  S.fac[0] = fac;
  S.coef[0] = coef;
  S.cpl[0] = cpl;
  S.top[0] = top;
  return solve_rows_set<C>(p, s, S, 1);
}

// Per-precision views of the slab buffers.
template <typename T>
struct SB;
template <>
struct SB<cplx> {
  static cplx* g(Slab& s) { return s.g; }
  static cplx* w(Slab& s) { return s.w; }
  static const cplx* fac(const Slab& s) { return s.fac; }
  static const cplx* coef(const Slab& s) { return s.coef; }
  static const cplx* cpl(const Slab& s) { return s.cpl; }
  static const cplx* tri(const ls_plan* p, const Slab& s) { return p->tri_ok ? s.tri : nullptr; }
  static cplx* work(ls_plan* p, int k) { return k ? p->slab_work2 : p->slab_work; }
  static cplx* elim(ls_plan* p) { return p->slab_elim; }
  static const cplx* top(const Slab& s) { return s.top; }
  static cplx* vtmp(ls_plan* p) { return p->vtmp; }
  static const cplx* mT(const Slab& s) { return s.mT; }
  static const cplx* mU(const Slab& s) { return s.mU; }
  static const cplx* mV(const Slab& s) { return s.mV; }
  static cplx* traces(ls_plan* p) { return p->traces; }
};
template <>
struct SB<fcplx> {
  static fcplx* g(Slab& s) { return s.g32; }
  static fcplx* w(Slab& s) { return s.w32; }
  static const fcplx* fac(const Slab& s) { return s.fac32; }
  static const fcplx* coef(const Slab& s) { return s.coef32; }
  static const fcplx* cpl(const Slab& s) { return s.cpl32; }
  static const fcplx* tri(const ls_plan* p, const Slab& s) { return p->tri_ok ? s.tri32 : nullptr; }
  static fcplx* work(ls_plan* p, int k) { return k ? p->slab_work32b : p->slab_work32; }
  static fcplx* elim(ls_plan* p) { return p->slab_elim32; }
  static const fcplx* top(const Slab& s) { return s.top32; }
  static fcplx* vtmp(ls_plan* p) { return p->vtmp32; }
  static const fcplx* mT(const Slab& s) { return s.mT32; }
  static const fcplx* mU(const Slab& s) { return s.mU32; }
  static const fcplx* mV(const Slab& s) { return s.mV32; }
  static fcplx* traces(ls_plan* p) { return p->traces32; }
};

// y = C_slab^{-1} g for B right-hand sides [B][n][q] (g untouched, y != g).
// One right-hand side runs the row-split out-of-place steps; several run
// the batched in-place steps on a copy.
template <typename T>
static ls_status solve_t(ls_plan* p, Slab& s, const T* g, T* y, int B) {
  if (B == 1)
    return solve_rows<T>(p, s, SB<T>::fac(s), SB<T>::coef(s), SB<T>::cpl(s), SB<T>::tri(p, s), SB<T>::top(s), g,
                         SB<T>::elim(p), y);
  LS_HIP(hipMemcpyAsync(y, g, (size_t)B * p->n * s.q * sizeof(T), hipMemcpyDeviceToDevice, p->stream));
  return solve_levels_b<T>(p, s, SB<T>::fac(s), SB<T>::coef(s), y, (size_t)p->n * s.q, B);
}

ls_status slab_solve(ls_plan* p, Slab& s, const cplx* g, cplx* y, int B) { return solve_t<cplx>(p, s, g, y, B); }
ls_status slab_solve(ls_plan* p, Slab& s, const fcplx* g, fcplx* y, int B) { return solve_t<fcplx>(p, s, g, y, B); }

// g^l gathered from g; with `up` set, plus the downward sweep's trace
// sources from the solution w of the layer above:
//   g^l += -delta_b C^l_{b,b+1} w^{l+1}(b+1) + delta_{b+1} C^l_{b+1,b} w^{l+1}(b)
template <typename T>
static ls_status gather(ls_plan* p, const Slab& s, const T* g, T* dst, int B, Slab* up, T* dst2 = nullptr) {
  const int n = p->n, tot = n * s.q;
  Inject A{}, Bj{};
  const T* sA = nullptr;
  if (up) {
    A = Inject{s.b - s.z0, +1, -1.0, up->q, s.b + 1 - up->z0};
    Bj = Inject{s.b + 1 - s.z0, -1, +1.0, up->q, s.b - up->z0};
    sA = SB<T>::w(*up);
  }
  // one right-hand side: the sources in the gather launch; many: a launch of their own
  const bool fuse = B == 1;
  if (!fuse && s.orient == 0)
    k_gather_h<T><<<dim3((n + kTI - 1) / kTI, (s.q + kTR - 1) / kTR, B), 256, 0, p->stream>>>(g, dst, n, s.q, s.z0,
                                                                                          s.a, s.b, dst2);
  else if (fuse && s.orient == 0 && !dst2)
    k_gather_h1<T><<<dim3((n + kTI1 - 1) / kTI1, (s.q + kTR - 1) / kTR), 128, 0, p->stream>>>(
        g, dst, n, s.q, s.z0, s.a, s.b, SB<T>::coef(s), A, Bj, sA);
  else
    k_gather<T><<<dim3((tot + 255) / 256, B), 256, 0, p->stream>>>(g, dst, n, s.q, s.z0, s.a, s.b, s.orient,
                                                                    SB<T>::coef(s), A, Bj, fuse ? sA : nullptr,
                                                                    dst2);
  if (sA && !fuse)
    k_inject<T><<<dim3((n + 255) / 256, B), 256, 0, p->stream>>>(dst, s.q, SB<T>::coef(s), n, A, Bj, sA, up->q,
                                                                  (const T*)nullptr, 0, 0, dst2);
  LS_HIP(hipGetLastError());
  return LS_OK;
}

// The layer rows of src (solution of layer s) into out; with `next` set,
// plus the upward sweep's trace sources for the next layer's right-hand
// side (v0 = src(a'-1), v1 = src(a') + w^{l'}(a') with a' the next layer's
// first line):
//   g^{l'} += -delta_a C_{a,a-1} v0 + delta_{a-1} C_{a-1,a} v1
template <typename T>
static ls_status scatter(ls_plan* p, const Slab& s, const T* src, T* out, bool acc, int B, Slab* next) {
  const bool fuse = B == 1;  // one right-hand side: the sources in the scatter launch
  const int n = p->n, tot = std::max(n * (s.b - s.a + 1), (next && fuse) ? n : 0);
  Inject A{}, Bj{};
  T* rhs = nullptr;
  const T* s2 = nullptr;
  int qr = 0, q2 = 0, r2 = 0;
  if (next) {
    Slab& nx = *next;
    A = Inject{nx.a - nx.z0, -1, -1.0, s.q, nx.a - 1 - s.z0};
    Bj = Inject{nx.a - 1 - nx.z0, +1, +1.0, s.q, nx.a - s.z0};
    rhs = SB<T>::g(nx);
    qr = nx.q;
    s2 = SB<T>::w(nx);
    q2 = nx.q;
    r2 = nx.a - nx.z0;
  }
  if (!fuse && s.orient == 0)
    k_scatter_h<T><<<dim3((n + kTI - 1) / kTI, (s.b - s.a + kTR) / kTR, B), 256, 0, p->stream>>>(
        src, out, n, s.q, s.z0, s.a, s.b, acc ? 1 : 0);
  else if (fuse && s.orient == 0)
    k_scatter_h1<T><<<dim3((n + kTI1 - 1) / kTI1, (s.b - s.a + kTR) / kTR), 128, 0, p->stream>>>(
        src, out, n, s.q, s.z0, s.a, s.b, acc ? 1 : 0, rhs, qr, next ? SB<T>::coef(*next) : nullptr, A, Bj, s2, q2,
        r2);
  else
    k_scatter<T><<<dim3((tot + 255) / 256, B), 256, 0, p->stream>>>(
        src, out, n, s.q, s.z0, s.a, s.b, s.orient, acc ? 1 : 0, fuse ? rhs : nullptr, qr,
        next ? SB<T>::coef(*next) : nullptr, A, Bj, s2, q2, r2);
  if (next && !fuse)
    k_inject<T><<<dim3((n + 255) / 256, B), 256, 0, p->stream>>>(rhs, qr, SB<T>::coef(*next), n, A, Bj, src, s.q,
                                                                  s2, q2, r2, (T*)nullptr);
  LS_HIP(hipGetLastError());
  return LS_OK;
}

// Alg. 1 for one right-hand side with the layers decoupled (the same linear
// operator): y^l = (C^l)^{-1} g^l for every layer; the traces the downward
// sweep passes, tau^l = R_tau w^l = R_tau y^l + mT^l tau^{l+1}, and the
// upward sweep's, sigma^l = R_sigma v^l + J tau^{l+1} = R_sigma y^l +
// (mU^l + J) tau^{l+1} + mV^l sigma^{l-1}, by two chains of dense products;
// then every layer's solve of g^l + E^l tau^{l+1} + F^l sigma^{l-1}, whose
// layer lines are Alg. 1's output.
// The per-layer work is batched over the layers: one launch gathers every
// g^l, one adds every layer's trace sources, one scatters every solution,
// and the independent solves run as one multi-slab chain per group of
// like slabs (the largest group on the plan's stream, the others on side
// streams forked from and joined back to it by events, so that a captured
// graph records them as parallel branches).

// Per-layer arguments of layers [l0, l0 + cnt): x = g^l, or the solution
// slot w^l when sol is set.
template <typename T>
static LayerSet<T> layer_set(ls_plan* p, std::vector<Slab>& S, int l0, int cnt, bool sol, const T* tau,
                             const T* sig) {
  const int L = (int)S.size(), N2 = 2 * p->n;
  LayerSet<T> ls{};
  for (int k = 0; k < cnt; ++k) {
    const int l = l0 + k;
    Slab& s = S[l];
    ls.x[k] = sol ? SB<T>::w(s) : SB<T>::g(s);
    ls.coef[k] = SB<T>::coef(s);
    ls.q[k] = s.q;
    ls.z0[k] = s.z0;
    ls.a[k] = s.a;
    ls.b[k] = s.b;
    ls.dn[k] = inj_down(s);
    ls.up[k] = inj_up(s);
    ls.tau[k] = (tau && l <= L - 2) ? tau + (size_t)(l + 1) * N2 : nullptr;
    ls.sig[k] = (sig && l >= 1) ? sig + (size_t)(l - 1) * N2 : nullptr;
  }
  return ls;
}

// w^l = (C^l)^{-1} g^l for every layer of one orientation, exact on the
// grid lines the next step reads: with `chains`, the lines a-1, a (layers
// l >= 1) and b, b+1 (layers l <= L-2) the trace chains read; without, the
// layer lines [a, b] the scatter reads.
template <typename T>
static ls_status solve_groups(ls_plan* p, int orient, bool chains) {
  std::vector<Slab>& S = p->slabs[orient];
  const std::vector<std::vector<int>>& G = p->dec_groups[orient];
  const size_t stride = (size_t)p->n * p->set_qmax;
  T* elim = static_cast<T*>(p->set_elim);
  auto run = [&](const std::vector<int>& grp) {
    SlabSet<T> ss{};
    for (size_t k = 0; k < grp.size(); ++k) {
      Slab& s = S[grp[k]];
      ss.g[k] = SB<T>::g(s);
      ss.t[k] = elim + (size_t)grp[k] * stride;
      ss.y[k] = SB<T>::w(s);
      ss.fac[k] = SB<T>::fac(s);
      ss.coef[k] = SB<T>::coef(s);
      ss.cpl[k] = SB<T>::cpl(s);
      ss.top[k] = SB<T>::top(s);
      const int l = grp[k], L = (int)S.size();
      const int want[4] = {l >= 1 ? s.a - s.z0 : -1, l >= 1 ? s.a - 1 - s.z0 : -1,
                           l <= L - 2 ? s.b - s.z0 : -1, l <= L - 2 ? s.b + 1 - s.z0 : -1};
      for (int u = 0; u < 4; ++u) ss.sel[k][u] = (want[u] >= 0 && want[u] < s.q) ? want[u] : -1;
      ss.lo[k] = s.a - s.z0;
      ss.hi[k] = s.b - s.z0 + 1;
      ss.tri[k] = SB<T>::tri(p, s);
    }
    return solve_rows_set<T>(p, S[grp[0]], ss, (int)grp.size(), chains ? ROWS_SEL : ROWS_RANGE);
  };
  constexpr int K = ls_plan::kSide;
  const int side = std::min((int)G.size() - 1, K);
  if (side > 0) {
    LS_HIP(hipEventRecord(p->side_fork, p->stream));
    for (int k = 0; k < side; ++k) LS_HIP(hipStreamWaitEvent(p->side[k], p->side_fork, 0));
  }
  // the largest group (the critical path) first: a captured graph replays
  // its branches' kernels in the order they were launched here, so a branch
  // launched later starts later
  ls_status st = run(G[0]);
  const hipStream_t main = p->stream;
  for (size_t gi = 1; gi < G.size() && st == LS_OK; ++gi) {
    p->stream = p->side[(gi - 1) % K];
    st = run(G[gi]);
  }
  p->stream = main;
  for (int k = 0; k < side; ++k) {
    LS_HIP(hipEventRecord(p->side_join[k], p->side[k]));
    LS_HIP(hipStreamWaitEvent(p->stream, p->side_join[k], 0));
  }
  return st;
}

template <typename T>
static ls_status sweep_decoupled_t(ls_plan* p, int orient, const T* g, T* v, bool accumulate) {
  std::vector<Slab>& S = p->slabs[orient];
  const int L = (int)S.size(), n = p->n, N2 = 2 * n;
  T* tau = SB<T>::traces(p);
  T* sig = tau + (size_t)L * N2;
  int qmax = 0, rmax = 0;
  for (const Slab& s : S) {
    qmax = std::max(qmax, s.q);
    rmax = std::max(rmax, s.b - s.a + 1);
  }
  for (int l0 = 0; l0 < L; l0 += kSet) {  // every g^l
    const int cnt = std::min(kSet, L - l0);
    const LayerSet<T> ls = layer_set<T>(p, S, l0, cnt, false, nullptr, nullptr);
    if (orient == 0)
      k_gather_set_h<T><<<dim3((n + 15) / 16, (qmax + kTR - 1) / kTR, cnt), 128, 0, p->stream>>>(g, ls, n);
    else
      k_gather_set_v<T><<<dim3((unsigned)(((size_t)n * qmax + 255) / 256), 1, cnt), 256, 0, p->stream>>>(g, ls, n);
  }
  LS_HIP(hipGetLastError());
  LS_TRY(solve_groups<T>(p, orient, true));  // the chains read four lines of each w^l
  // the traces: tau^l = R_tau y^l + mT^l tau^{l+1} from the top layer down
  // (a chain); sigma0^l = R_sigma y^l + (mU^l + J) tau^{l+1} for every
  // layer at once; sigma^l = sigma0^l + mV^l sigma^{l-1} upwards (a chain)
  const unsigned rows4 = (unsigned)((N2 + 3) / 4);
  for (int l = L - 1; l >= 1; --l) {
    Slab& s = S[l];
    const bool m = l <= L - 2;
    TraceSet<T> ts{};
    ts.out[0] = tau + (size_t)l * N2;
    ts.y[0] = SB<T>::w(s);
    ts.M[0] = m ? SB<T>::mT(s) : nullptr;
    ts.x[0] = m ? tau + (size_t)(l + 1) * N2 : nullptr;
    ts.q[0] = s.q;
    ts.r0[0] = s.a - s.z0;
    ts.r1[0] = s.a - 1 - s.z0;
    k_trace_set<T, 4><<<dim3(N2, 1), 256, 0, p->stream>>>(ts, n, 0);
  }
  for (int l0 = 0; l0 <= L - 2; l0 += kSet) {
    const int cnt = std::min(kSet, L - 1 - l0);
    TraceSet<T> ts{};
    for (int k = 0; k < cnt; ++k) {
      Slab& s = S[l0 + k];
      ts.out[k] = sig + (size_t)(l0 + k) * N2;
      ts.y[k] = SB<T>::w(s);
      ts.M[k] = SB<T>::mU(s);
      ts.x[k] = tau + (size_t)(l0 + k + 1) * N2;
      ts.q[k] = s.q;
      ts.r0[k] = s.b - s.z0;
      ts.r1[k] = s.b + 1 - s.z0;
    }
    k_trace_set<T, 1><<<dim3(rows4, cnt), 256, 0, p->stream>>>(ts, n, 1);
  }
  for (int l = 1; l <= L - 2; ++l) {
    TraceSet<T> ts{};
    ts.out[0] = sig + (size_t)l * N2;
    ts.base[0] = ts.out[0];
    ts.M[0] = SB<T>::mV(S[l]);
    ts.x[0] = sig + (size_t)(l - 1) * N2;
    k_trace_set<T, 4><<<dim3(N2, 1), 256, 0, p->stream>>>(ts, n, 0);
  }
  for (int l0 = 0; l0 < L; l0 += kSet) {  // every layer's trace sources into g^l
    const int cnt = std::min(kSet, L - l0);
    k_inject_set<T><<<dim3((n + 255) / 256, 1, cnt), 256, 0, p->stream>>>(
        layer_set<T>(p, S, l0, cnt, false, tau, sig), n);
  }
  LS_HIP(hipGetLastError());
  LS_TRY(solve_groups<T>(p, orient, false));  // the chains have read w^l: it takes the final solutions
  for (int l0 = 0; l0 < L; l0 += kSet) {  // their layer lines into v
    const int cnt = std::min(kSet, L - l0);
    const LayerSet<T> ls = layer_set<T>(p, S, l0, cnt, true, nullptr, nullptr);
    if (orient == 0)
      k_scatter_set_h<T><<<dim3((n + 15) / 16, (rmax + kTR - 1) / kTR, cnt), 128, 0, p->stream>>>(
          v, ls, n, accumulate ? 1 : 0);
    else
      k_scatter_set_v<T><<<dim3((unsigned)(((size_t)n * rmax + 255) / 256), 1, cnt), 256, 0, p->stream>>>(
          v, ls, n, accumulate ? 1 : 0);
  }
  LS_HIP(hipGetLastError());
  return LS_OK;
}

// Alg. 1 (Gauss-Seidel polarized traces) on layers of one orientation, for
// B right-hand sides at once.  v receives the concatenated layer solutions
// (or has them added).
template <typename T>
static ls_status sweep_t(ls_plan* p, int orient, const T* g, T* v, bool accumulate, int B) {
  std::vector<Slab>& S = p->slabs[orient];
  const int L = (int)S.size();
  if (B == 1 && L >= 2 && p->opt.sweep == LS_SWEEP_DECOUPLED && SB<T>::traces(p))
    return sweep_decoupled_t<T>(p, orient, g, v, accumulate);
  // downward sweep: l = L-1 .. 0 (gather with the trace sources of w^{l+1})
  for (int l = L - 1; l >= 0; --l) {
    Slab& s = S[l];
    if (B == 1) {
      LS_TRY(gather<T>(p, s, g, SB<T>::g(s), B, l != L - 1 ? &S[l + 1] : nullptr));
      LS_TRY(solve_t<T>(p, s, SB<T>::g(s), SB<T>::w(s), B));
    } else {
      // g^l is kept for the upward sweep; the batched steps run in place on
      // a second copy that the gather writes alongside it
      LS_TRY(gather<T>(p, s, g, SB<T>::g(s), B, l != L - 1 ? &S[l + 1] : nullptr, SB<T>::w(s)));
      LS_TRY(solve_levels_b<T>(p, s, SB<T>::fac(s), SB<T>::coef(s), SB<T>::w(s), (size_t)p->n * s.q, B));
    }
  }
  // upward sweep: l = 0 .. L-1; scattering v^{l-1} also adds its trace
  // sources to g^l
  T* vprev = nullptr;
  for (int l = 0; l < L; ++l) {
    Slab& s = S[l];
    T* vcur;
    if (l == 0) {
      vcur = SB<T>::w(s);  // g^0 is unchanged: v^0 = w^0
    } else if (B == 1) {
      vcur = SB<T>::work(p, vprev == SB<T>::work(p, 0) ? 1 : 0);
      LS_TRY(scatter<T>(p, S[l - 1], vprev, v, accumulate, B, &s));
      LS_TRY(solve_t<T>(p, s, SB<T>::g(s), vcur, B));
    } else {
      // g^l is not needed after this solve: the batched steps run in place
      vcur = SB<T>::g(s);
      LS_TRY(scatter<T>(p, S[l - 1], vprev, v, accumulate, B, &s));
      LS_TRY(solve_levels_b<T>(p, s, SB<T>::fac(s), SB<T>::coef(s), vcur, (size_t)p->n * s.q, B));
    }
    if (l == L - 1) LS_TRY(scatter<T>(p, s, vcur, v, accumulate, B, nullptr));
    vprev = vcur;
  }
  return LS_OK;
}

ls_status sweep_apply(ls_plan* p, int orient, const cplx* g, cplx* v, bool accumulate, int B) {
  return sweep_t<cplx>(p, orient, g, v, accumulate, B);
}
ls_status sweep_apply(ls_plan* p, int orient, const fcplx* g, fcplx* v, bool accumulate, int B) {
  return sweep_t<fcplx>(p, orient, g, v, accumulate, B);
}

// Alg. 2: u1 = Prec_H(g); e = g - C u1; u2 = Prec_V(e); v = u1 + u2.
template <typename T>
static ls_status bidir_t(ls_plan* p, const T* g, T* v, int B) {
  T* e = SB<T>::vtmp(p);
  LS_TRY(sweep_t<T>(p, 0, g, v, false, B));
  LS_TRY(stencil_residual_C(p, g, v, e, B));
  LS_TRY(sweep_t<T>(p, 1, e, v, true, B));
  return LS_OK;
}

ls_status bidirectional_apply(ls_plan* p, const cplx* g, cplx* v, int B) { return bidir_t<cplx>(p, g, v, B); }
ls_status bidirectional_apply(ls_plan* p, const fcplx* g, fcplx* v, int B) { return bidir_t<fcplx>(p, g, v, B); }

// ------------------------------------------------- allocation-free slab solve
// The single-right-hand-side slab solve with its scratch -- the eliminated
// right-hand sides t, and the copies of b and x an FP32 plan or an in-place
// call needs -- in a file-scope device array instead of plan memory, for
// callers that cannot allocate (graph capture, serving loops).  Each GPU
// holds its own copy of the array for the life of the process; host code
// never uses the array's name, only the device address taken once per
// device by static_scratch_init (at plan creation, with the device current).
// Calls on one GPU share the array: they must not overlap.
constexpr size_t kScratchBytes = (size_t)6 << 20;  // 2 * n * q * 16 B at n = 2048, q = 96
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
namespace {
constexpr int kScratchDevices = 64;
void* g_scratch_dev[kScratchDevices];
std::mutex g_scratch_mu;

__global__ void k_up_copy(const fcplx* __restrict__ a, cplx* __restrict__ b, size_t cnt) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < cnt) b[i] = cmk((double)a[i].x, (double)a[i].y);
}
}  // namespace

size_t static_scratch_bytes() { return kScratchBytes; }

ls_status static_scratch_init(int device) {
  if (device < 0 || device >= kScratchDevices) {
    ls_set_error("static scratch: device index out of range");
    return LS_EUNSUPPORTED;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_dev[device]) return LS_OK;
  void* ptr = nullptr;
  LS_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
  if (!ptr) {
    ls_set_error("static scratch: hipGetSymbolAddress returned a null address");
    return LS_EDEVICE;
  }
  g_scratch_dev[device] = ptr;
  return LS_OK;
}

ls_status slab_solve_noalloc(ls_plan* p, Slab& s, const cplx* b, cplx* x) {
  void* base = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (p->device >= 0 && p->device < kScratchDevices) base = g_scratch_dev[p->device];
  }
  if (!base) {
    ls_set_error("ls_slab_solve_noalloc: static scratch of this device not set up");
    return LS_EDEVICE;
  }
  const size_t cnt = (size_t)p->n * s.q;
  const unsigned blocks = (unsigned)((cnt + 255) / 256);
  if (p->fp32) {
    if (3 * cnt * sizeof(fcplx) > kScratchBytes) {
      ls_set_error("ls_slab_solve_noalloc: slab of " + std::to_string(cnt) + " unknowns exceeds the " +
                   std::to_string(kScratchBytes) + "-byte static scratch");
      return LS_EINVAL;
    }
    fcplx* gi = reinterpret_cast<fcplx*>(base);
    fcplx* yo = gi + cnt;
    fcplx* t = yo + cnt;
    k_down_copy<<<blocks, 256, 0, p->stream>>>(b, gi, cnt);
    LS_TRY(solve_rows<fcplx>(p, s, s.fac32, s.coef32, s.cpl32, SB<fcplx>::tri(p, s), s.top32, gi, t, yo));
    k_up_copy<<<blocks, 256, 0, p->stream>>>(yo, x, cnt);
    LS_HIP(hipGetLastError());
    return LS_OK;
  }
  const bool inplace = b == x;
  if ((inplace ? 2 : 1) * cnt * sizeof(cplx) > kScratchBytes) {
    ls_set_error("ls_slab_solve_noalloc: slab of " + std::to_string(cnt) + " unknowns exceeds the " +
                 std::to_string(kScratchBytes) + "-byte static scratch");
    return LS_EINVAL;
  }
  cplx* t = reinterpret_cast<cplx*>(base);
  const cplx* g = b;
  if (inplace) {
    cplx* gi = t + cnt;
    LS_HIP(hipMemcpyAsync(gi, b, cnt * sizeof(cplx), hipMemcpyDeviceToDevice, p->stream));
    g = gi;
  }
  return solve_rows<cplx>(p, s, s.fac, s.coef, s.cpl, SB<cplx>::tri(p, s), s.top, g, t, x);
}
