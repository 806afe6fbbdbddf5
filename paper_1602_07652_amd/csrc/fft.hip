// Zero-padded 2-D FFT convolution: the operator H = I + omega^2 G D.
//
// Section 2: G is embedded in a Toeplitz (circulant) matrix and applied
// with the FFT; Section 4.2: the cost of H is dominated by the FFT.
//
// Layout on the device (FP64 complex):
//   v, y           [batch][n][n]          x fastest
//   X (work)       [batch][P/T][n][T]     row spectra, tiled by T columns
//                                         (T = 8 for FP64, 16 for FP32: one
//                                         128-byte line) so every row pass
//                                         moves whole lines and a column pass
//                                         reads up to T adjacent columns
//   spec           [P/2+1][P/2+1]         quarter of FFT2(circulant w),
//                                         scaled by omega^2 / P^2
// Passes (one HBM round trip of the n x P intermediate each way):
//   K1 rows:    X_j = FFT_P(pad(m_j . v_j))                 (pruned input)
//   K2 columns: Y_c = first n of IFFT_P(S_c . FFT_P(pad(X_c)))
//   K3 rows:    y_j = a v_j + b (first n of IFFT_P(Y_j))    (pruned output)
// Each transform is a radix-4 Stockham FFT (one radix-2 pass first when
// log2 P is odd) done in LDS, with the twiddles read from a P-entry table.
// Everything is templated on the complex type (double2: FP64 path; float2:
// the FP32 operator of the refinement loop).
#include "ls_internal.h"

#include <algorithm>
#include <type_traits>
#include <cmath>

namespace {

template <typename T>
struct Tile {
  static constexpr int W = 128 / (int)sizeof(T);  // columns per 128-byte line
};

template <typename T, bool INV>
__device__ __forceinline__ void radix4(T& a0, T& a1, T& a2, T& a3) {
  const T t0 = tadd(a0, a2), t1 = tsub(a0, a2), t2 = tadd(a1, a3), t3 = tsub(a1, a3);
  // forward: X1 = t1 - i t3, X3 = t1 + i t3 ; inverse: conjugate roots
  T it3;
  if (INV) { it3.x = -t3.y; it3.y = t3.x; } else { it3.x = t3.y; it3.y = -t3.x; }
  a0 = tadd(t0, t2);
  a2 = tsub(t0, t2);
  a1 = tadd(t1, it3);
  a3 = tsub(t1, it3);
}

// COUNT transforms of length 2^LOGN held in LDS at buf + c*STRIDE, done by
// NT threads in place (every thread keeps its butterflies in registers
// between the read and the write of a pass).
template <typename T, int LOGN, int COUNT, int STRIDE, int NT, bool INV>
__device__ __forceinline__ void fft_lds(T* buf, const T* __restrict__ tw, int tid) {
  constexpr int N = 1 << LOGN;
  if constexpr ((LOGN & 1) != 0) {
    constexpr int NB = COUNT * (N / 2);
    constexpr int K = (NB + NT - 1) / NT;
    T a[K], b[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int bi = tid + k * NT;
      if (bi < NB) {
        const int c = bi / (N / 2), j = bi % (N / 2);
        a[k] = buf[c * STRIDE + j];
        b[k] = buf[c * STRIDE + j + N / 2];
      }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int bi = tid + k * NT;
      if (bi < NB) {
        const int c = bi / (N / 2), j = bi % (N / 2);
        buf[c * STRIDE + 2 * j] = tadd(a[k], b[k]);
        buf[c * STRIDE + 2 * j + 1] = tsub(a[k], b[k]);
      }
    }
    __syncthreads();
  }
  constexpr int NS0 = (LOGN & 1) ? 2 : 1;
  constexpr int NB = COUNT * (N / 4);
  constexpr int K = (NB + NT - 1) / NT;
#pragma unroll
  for (int Ns = NS0; Ns < N; Ns *= 4) {
    T v[K][4];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int bi = tid + k * NT;
      if (bi < NB) {
        const int c = bi / (N / 4), j = bi % (N / 4);
        const T* src = buf + c * STRIDE + j;
        v[k][0] = src[0];
        v[k][1] = src[N / 4];
        v[k][2] = src[2 * (N / 4)];
        v[k][3] = src[3 * (N / 4)];
        if (Ns > 1) {
          const int jm = j & (Ns - 1);
          const int st = N / (Ns * 4);
          T w1 = tw[jm * st], w2 = tw[2 * jm * st], w3 = tw[3 * jm * st];
          if (INV) { w1.y = -w1.y; w2.y = -w2.y; w3.y = -w3.y; }
          v[k][1] = tmul(v[k][1], w1);
          v[k][2] = tmul(v[k][2], w2);
          v[k][3] = tmul(v[k][3], w3);
        }
        radix4<T, INV>(v[k][0], v[k][1], v[k][2], v[k][3]);
      }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int bi = tid + k * NT;
      if (bi < NB) {
        const int c = bi / (N / 4), j = bi % (N / 4);
        const int jm = j & (Ns - 1);
        T* dst = buf + c * STRIDE + (j / Ns) * Ns * 4 + jm;
        dst[0] = v[k][0];
        dst[Ns] = v[k][1];
        dst[2 * Ns] = v[k][2];
        dst[3 * Ns] = v[k][3];
      }
    }
    __syncthreads();
  }
}

// Row passes: COUNT rows of length N per workgroup of NT threads.
template <int LOGN>
struct RowCfg {
  static constexpr int N = 1 << LOGN;
  static constexpr int NT = (N / 4 > 256) ? N / 4 : 256;
  static constexpr int COUNT = NT * 4 / N;
};

// Column pass: CPW adjacent columns per workgroup (<= 128 KB of LDS).
// Variant V halves CPW V times (the autotuner picks V per plan).
template <typename T, int LOGN, int V = 0>
struct ColCfg {
  static constexpr int N = 1 << LOGN;
  static constexpr int LIM = (131072 / (int)sizeof(T)) / N;
  static constexpr int CPW0 = (LIM < Tile<T>::W) ? LIM : Tile<T>::W;
  static constexpr int CPW = (CPW0 >> V) > 0 ? (CPW0 >> V) : 1;
  static constexpr int NT0 = CPW * N / 4;
  static constexpr int NT = NT0 > 1024 ? 1024 : (NT0 < 64 ? 64 : NT0);
  static constexpr int STRIDE = N + 1;  // pad: adjacent columns in different banks
};
constexpr int kRowHalf = 1;  // row passes: half tile (two workgroups per CU)
constexpr int kColVariants = kFftVariants;  // 0, 1: radix-16 register passes, full / half tile; 2-4: LDS passes V = 0..2;
                                  // 5: radix-8 register passes; 6: even / odd half-length transforms, one
                                  // column per workgroup; 7: as 0 with a quarter tile (P = 1024..4096;
                                  // smaller P: LDS passes)

template <typename T>
__device__ __forceinline__ size_t tiled(int b, int n, int N, int j, int kx) {
  constexpr int W = Tile<T>::W;
  return (size_t)b * n * N + ((size_t)(kx / W) * n + j) * W + (kx % W);
}

// K1: X = FFT_rows(pad(m . v)).
template <typename T, typename R, int LOGN>
__global__ __launch_bounds__(RowCfg<LOGN>::NT) void k_rows_fwd(const T* __restrict__ v,
                                                             const R* __restrict__ m,
                                                             T* __restrict__ X,
                                                             const T* __restrict__ tw, int n,
                                                             int total_rows) {
  using C = RowCfg<LOGN>;
  constexpr int N = C::N;
  extern __shared__ unsigned char lds_raw[];
  T* buf = reinterpret_cast<T*>(lds_raw);
  const int tid = threadIdx.x;
  const int row0 = blockIdx.x * C::COUNT;
  for (int e = tid; e < C::COUNT * N; e += C::NT) {
    const int c = e / N, i = e % N;
    const int row = row0 + c;
    T val = tmk<T>(0, 0);
    if (row < total_rows && i < n) {
      const int j = row % n;
      const T vv = v[(size_t)row * n + i];
      const R mm = m[(size_t)j * n + i];
      val.x = vv.x * mm;
      val.y = vv.y * mm;
    }
    buf[e] = val;
  }
  __syncthreads();
  fft_lds<T, LOGN, C::COUNT, N, C::NT, false>(buf, tw, tid);
  for (int e = tid; e < C::COUNT * N; e += C::NT) {
    const int c = e / N, kx = e % N;
    const int row = row0 + c;
    if (row < total_rows) X[tiled<T>(row / n, n, N, row % n, kx)] = buf[e];
  }
}

// Maps the hardware workgroup id so that consecutive logical ids run on
// the same XCD (ids are dispatched round-robin over the 8 XCDs): the
// column groups that share 128-byte lines then share one L2.
__device__ __forceinline__ int xcd_remap(int id, int total) {
  const int per = total / 8;
  if (per == 0 || id >= per * 8) return id;
  return (id % 8) * per + id / 8;
}

// Column group g -> (right-hand side b, group cg).  The S = W / CPW groups
// that share the 128-byte lines of one tile of W columns are consecutive,
// then come the other right-hand sides of that tile, then the mirror tile
// (columns N - kx read the same rows of the quarter spectrum as kx): the run
// of groups one XCD takes reads each line and each spectrum row into its L2
// once.  N / W is even.
__device__ __forceinline__ void col_group(int g, int G, int total, int S, int& b, int& cg) {
  const int B = total / G, M = G / S;
  const int P = g / (S * B), rem = g - P * S * B;
  b = rem / S;
  const int tile = (P & 1) ? M - 1 - (P >> 1) : (P >> 1);
  cg = tile * S + (rem - b * S);
}

// K2: per column c of X: FFT, multiply by the spectrum, IFFT, keep n.
template <typename T, int LOGN, int V>
__global__ __launch_bounds__((ColCfg<T, LOGN, V>::NT)) void k_cols_conv(T* __restrict__ X,
                                                                    const T* __restrict__ spec,
                                                                    const T* __restrict__ tw, int n,
                                                                    int ss, int groups_per_rhs,
                                                                    int total_groups) {
  using C = ColCfg<T, LOGN, V>;
  constexpr int N = C::N, CPW = C::CPW, S = C::STRIDE, W = Tile<T>::W;
  extern __shared__ unsigned char lds_raw[];
  T* buf = reinterpret_cast<T*>(lds_raw);
  const int tid = threadIdx.x;
  const int g = xcd_remap(blockIdx.x, total_groups);
  int b, cg;
  col_group(g, groups_per_rhs, total_groups, W / CPW, b, cg);
  const int c0 = cg * CPW;
  T* Xb = X + (size_t)b * n * N + (size_t)(c0 / W) * n * W + (c0 % W);
  for (int e = tid; e < CPW * n; e += C::NT) {
    const int j = e / CPW, cc = e % CPW;
    buf[cc * S + j] = Xb[(size_t)j * W + cc];
  }
  for (int e = tid; e < CPW * (N - n); e += C::NT) {
    const int cc = e / (N - n), j = n + e % (N - n);
    buf[cc * S + j] = tmk<T>(0, 0);
  }
  __syncthreads();
  fft_lds<T, LOGN, CPW, S, C::NT, false>(buf, tw, tid);
  for (int e = tid; e < CPW * N; e += C::NT) {
    const int cc = e / N, ky = e % N;
    const int kx = c0 + cc;
    const int kxq = kx <= N / 2 ? kx : N - kx;
    const int kyq = ky <= N / 2 ? ky : N - ky;
    buf[cc * S + ky] = tmul(buf[cc * S + ky], spec[(size_t)kxq * ss + kyq]);
  }
  __syncthreads();
  fft_lds<T, LOGN, CPW, S, C::NT, true>(buf, tw, tid);
  for (int e = tid; e < CPW * n; e += C::NT) {
    const int j = e / CPW, cc = e % CPW;
    Xb[(size_t)j * W + cc] = buf[cc * S + j];
  }
}

// ---------------------------------------------------------------------
// K2 with register-resident radix-16/8 passes (P = 1024, 2048, 4096).
// Each column is transformed by Stockham passes whose radix-R butterflies
// live in registers (R = 16 or 8 points per butterfly), so a transform is
// 3 passes with 2 exchanges through LDS instead of 6 radix-2/4 passes.
// The forward transform starts from global memory (only the n nonzero
// inputs are loaded) and ends in natural order in registers; the spectrum
// multiply happens there, and the inverse transform starts from the same
// registers (its first radix equals the forward's last, so each thread
// already holds the element set its first butterfly needs); its last pass
// writes only the n outputs that are kept.  LDS rows are padded by one
// element every 16 so strided butterfly reads and writes spread over the
// banks.

// cos / sin of 2 pi m / 16, m = 0..15
__device__ __constant__ const double kC16[16] = {
    1.0, 0.92387953251128675613, 0.70710678118654752440, 0.38268343236508977173,
    0.0, -0.38268343236508977173, -0.70710678118654752440, -0.92387953251128675613,
    -1.0, -0.92387953251128675613, -0.70710678118654752440, -0.38268343236508977173,
    0.0, 0.38268343236508977173, 0.70710678118654752440, 0.92387953251128675613};
__device__ __constant__ const double kS16[16] = {
    0.0, 0.38268343236508977173, 0.70710678118654752440, 0.92387953251128675613,
    1.0, 0.92387953251128675613, 0.70710678118654752440, 0.38268343236508977173,
    0.0, -0.38268343236508977173, -0.70710678118654752440, -0.92387953251128675613,
    -1.0, -0.92387953251128675613, -0.70710678118654752440, -0.38268343236508977173};

// e^{-+2 pi i m / 16} (forward: minus)
template <typename T, bool INV>
__device__ __forceinline__ T w16(int m) {
  return tmk<T>(kC16[m & 15], INV ? kS16[m & 15] : -kS16[m & 15]);
}

// In-register DFTs, natural order in and out.
template <typename T, bool INV>
__device__ __forceinline__ void dft8(T* a) {
  T e0 = a[0], e1 = a[2], e2 = a[4], e3 = a[6];
  T o0 = a[1], o1 = a[3], o2 = a[5], o3 = a[7];
  radix4<T, INV>(e0, e1, e2, e3);
  radix4<T, INV>(o0, o1, o2, o3);
  const T E[4] = {e0, e1, e2, e3};
  T O[4] = {o0, o1, o2, o3};
#pragma unroll
  for (int k = 1; k < 4; ++k) O[k] = tmul(O[k], w16<T, INV>(2 * k));
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    a[k] = tadd(E[k], O[k]);
    a[k + 4] = tsub(E[k], O[k]);
  }
}

template <typename T, bool INV>
__device__ __forceinline__ void dft16(T* a) {
  // n = 4 n1 + n2: inner DFT over n1 for each n2, twiddle W16^{n2 k1},
  // outer DFT over n2: X[k1 + 4 k2]
  T y[4][4];
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) {
    T b0 = a[n2], b1 = a[n2 + 4], b2 = a[n2 + 8], b3 = a[n2 + 12];
    radix4<T, INV>(b0, b1, b2, b3);
    y[n2][0] = b0;
    y[n2][1] = n2 ? tmul(b1, w16<T, INV>(n2)) : b1;
    y[n2][2] = n2 ? tmul(b2, w16<T, INV>(2 * n2)) : b2;
    y[n2][3] = n2 ? tmul(b3, w16<T, INV>(3 * n2)) : b3;
  }
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    T c0 = y[0][k1], c1 = y[1][k1], c2 = y[2][k1], c3 = y[3][k1];
    radix4<T, INV>(c0, c1, c2, c3);
    a[k1] = c0;
    a[k1 + 4] = c1;
    a[k1 + 8] = c2;
    a[k1 + 12] = c3;
  }
}

template <typename T, int R, bool INV>
__device__ __forceinline__ void dft_r(T* a) {
  if constexpr (R == 16) dft16<T, INV>(a);
  else if constexpr (R == 8) dft8<T, INV>(a);
  else radix4<T, INV>(a[0], a[1], a[2], a[3]);
}

// Stockham pass on one butterfly j (span NS, radix R, length N): inputs
// x[j + r N/R] twiddled by W_{NS R}^{r (j mod NS)}, outputs to
// (j - k) R + k + r NS with k = j mod NS.
// The powers w^r, r < R, of the butterfly's twiddle w = W_{NS R}^k come
// from the table at r = 1, 2, 4, 8 and one complex product each for the
// others (at most one extra rounding).
template <typename T, int N, int R, int NS, bool INV>
__device__ __forceinline__ void twiddle_r(T* a, int j, const T* __restrict__ tw) {
  if constexpr (NS > 1) {
    const int k = j & (NS - 1);
    constexpr int st = N / (NS * R);
    T w[R];
    w[1] = tw[k * st];
    w[2] = tw[2 * k * st];
    w[3] = tmul(w[2], w[1]);
    if constexpr (R >= 8) {
      w[4] = tw[4 * k * st];
      w[5] = tmul(w[4], w[1]);
      w[6] = tmul(w[4], w[2]);
      w[7] = tmul(w[4], w[3]);
    }
    if constexpr (R == 16) {
      w[8] = tw[8 * k * st];
#pragma unroll
      for (int r = 9; r < 16; ++r) w[r] = tmul(w[8], w[r - 8]);
    }
#pragma unroll
    for (int r = 1; r < R; ++r) {
      T x = w[r];
      if (INV) x.y = -x.y;
      a[r] = tmul(a[r], x);
    }
  }
}

__device__ __forceinline__ int lpad(int i) { return i + (i >> 4); }

// radices of the forward transform; the inverse uses them reversed
template <int LOGN> struct RegPlan;
template <> struct RegPlan<10> { static constexpr int R0 = 16, R1 = 8, R2 = 8; };
template <> struct RegPlan<11> { static constexpr int R0 = 16, R1 = 16, R2 = 8; };
template <> struct RegPlan<12> { static constexpr int R0 = 16, R1 = 16, R2 = 16; };

// Columns per workgroup: the most whose padded LDS columns fit in 150 KB
// with at most 1024 threads (one radix-16 butterfly each); variants H = 1, 2
// halve and quarter it.
template <typename T, int LOGN, int H = 0>
struct RegCfg {
  static constexpr int N = 1 << LOGN;
  // padded column in LDS: one element per 16, and a stride of 2 (mod 16)
  // elements between columns, so the lanes of the global-memory passes
  // (columns fastest) and of the LDS-only passes (butterflies fastest) both
  // fall in distinct banks
  static constexpr int ROW = N + N / 16 + 2;
  static constexpr int fit(int c) {
    return (c * 2 * ROW * (int)sizeof(T) <= 153600 && c * 2 * N / 16 <= 1024) ? fit(2 * c) : c;
  }
  // at most one tile of W columns (the group's columns share its rows)
  static constexpr int C0 = fit(1) < Tile<T>::W ? fit(1) : Tile<T>::W;
  static constexpr int CPW = (C0 >> H) > 0 ? (C0 >> H) : 1;
  static constexpr int NT = CPW * N / 16;
  static_assert(CPW <= Tile<T>::W, "a column group stays inside one tile");
  static constexpr size_t lds() { return (size_t)CPW * ROW * sizeof(T); }
};

// Butterfly bi of a pass -> (column, butterfly index): columns fastest, so
// the lanes of a wave that touch global memory pair up within lines.
template <int CPW>
__device__ __forceinline__ void bsplit(int bi, int& cc, int& j) {
  cc = bi % CPW;
  j = bi / CPW;
}

// Middle pass: LDS -> registers -> LDS.
template <typename T, int N, int R, int NS, int CPW, int ROW, int NT, bool INV, int TN = N>
__device__ __forceinline__ void reg_pass(T* buf, const T* __restrict__ tw, int tid) {
  constexpr int NB = N / R, PER = CPW * NB / NT;
  T a[PER][R];
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int bi = tid + NT * q, cc = bi / NB, j = bi % NB;  // butterflies fastest
#pragma unroll
    for (int r = 0; r < R; ++r) a[q][r] = buf[cc * ROW + lpad(j + r * NB)];
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int bi = tid + NT * q, cc = bi / NB, j = bi % NB;
    twiddle_r<T, TN, R, NS, INV>(a[q], j, tw);
    dft_r<T, R, INV>(a[q]);
    const int k = j & (NS - 1);
#pragma unroll
    for (int r = 0; r < R; ++r) buf[cc * ROW + lpad((j - k) * R + k + r * NS)] = a[q][r];
  }
  __syncthreads();
}

// One group of CPW columns of K2.  Pass 0 takes its inputs (elements
// j + r N/R0 of column cc, zero past n) from registers, so that a persistent
// workgroup can load the next group while it transforms this one.
template <typename T, int LOGN, int H>
__device__ __forceinline__ void cols_reg_load(const T* __restrict__ Xb, T* a, int tid, int n) {
  using C = RegCfg<T, LOGN, H>;
  constexpr int N = C::N, CPW = C::CPW, W = Tile<T>::W, R0 = RegPlan<LOGN>::R0, NB = N / R0;
  int cc, j;
  bsplit<CPW>(tid, cc, j);
#pragma unroll
  for (int r = 0; r < R0; ++r) {
    const int e = j + r * NB;
    a[r] = e < n ? Xb[(size_t)e * W + cc] : tmk<T>(0, 0);
  }
}

template <typename T, int LOGN, int H>
__device__ __forceinline__ T* cols_reg_base(T* X, int g, int groups_per_rhs, int total, int n, int& c0) {
  constexpr int N = 1 << LOGN, CPW = RegCfg<T, LOGN, H>::CPW, W = Tile<T>::W;
  int b, cg;
  col_group(g, groups_per_rhs, total, W / CPW, b, cg);
  c0 = cg * CPW;
  return X + (size_t)b * n * N + (size_t)(c0 / W) * n * W + (c0 % W);
}

template <typename T, int LOGN, int H>
__device__ __forceinline__ void cols_reg_group(T* __restrict__ Xb, int c0, T* a0, T* buf,
                                               const T* __restrict__ spec, const T* __restrict__ tw,
                                               int n, int ss, int tid) {
  using C = RegCfg<T, LOGN, H>;
  using PL = RegPlan<LOGN>;
  constexpr int N = C::N, CPW = C::CPW, ROW = C::ROW, W = Tile<T>::W, NT = C::NT;
  constexpr int R0 = PL::R0, R1 = PL::R1, R2 = PL::R2;
  // forward pass 0 (radix 16, span 1) on the loaded column elements
  {
    int cc, j;
    bsplit<CPW>(tid, cc, j);
    dft_r<T, R0, false>(a0);
#pragma unroll
    for (int r = 0; r < R0; ++r) buf[cc * ROW + lpad(j * R0 + r)] = a0[r];
  }
  __syncthreads();
  reg_pass<T, N, R1, R0, CPW, ROW, NT, false>(buf, tw, tid);
  // forward last pass (span R0 R1), spectrum multiply and inverse first pass
  // in registers: butterfly j holds elements j + r N/R2 in natural order
  {
    constexpr int NB = N / R2, NS = R0 * R1, PER = CPW * NB / NT;
    T a[PER][R2];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int bi = tid + NT * q, cc = bi / NB, j = bi % NB;  // butterflies fastest (LDS, spectrum)
#pragma unroll
      for (int r = 0; r < R2; ++r) a[q][r] = buf[cc * ROW + lpad(j + r * NB)];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int bi = tid + NT * q, cc = bi / NB, j = bi % NB;  // butterflies fastest (LDS, spectrum)
      twiddle_r<T, N, R2, NS, false>(a[q], j, tw);
      dft_r<T, R2, false>(a[q]);
      const int kx = c0 + cc;
      const int kxq = kx <= N / 2 ? kx : N - kx;
#pragma unroll
      for (int r = 0; r < R2; ++r) {
        const int ky = j + r * NB;
        const int kyq = ky <= N / 2 ? ky : N - ky;
        a[q][r] = tmul(a[q][r], spec[(size_t)kxq * ss + kyq]);
      }
      dft_r<T, R2, true>(a[q]);  // inverse pass 0 (span 1)
#pragma unroll
      for (int r = 0; r < R2; ++r) buf[cc * ROW + lpad(j * R2 + r)] = a[q][r];
    }
  }
  __syncthreads();
  reg_pass<T, N, R1, R2, CPW, ROW, NT, true>(buf, tw, tid);
  // inverse last pass (radix R0, span R2 R1): natural order, keep n outputs
  {
    constexpr int NB = N / R0, NS = R2 * R1;
    int cc, j;
    bsplit<CPW>(tid, cc, j);
    T a[R0];
#pragma unroll
    for (int r = 0; r < R0; ++r) a[r] = buf[cc * ROW + lpad(j + r * NB)];
    twiddle_r<T, N, R0, NS, true>(a, j, tw);
    dft_r<T, R0, true>(a);
#pragma unroll
    for (int r = 0; r < R0; ++r) {
      const int e = j + r * NB;
      if (e < n) Xb[(size_t)e * W + cc] = a[r];
    }
  }
}

template <typename T, int LOGN, int H>
__global__ __launch_bounds__((RegCfg<T, LOGN, H>::NT)) void k_cols_reg(T* __restrict__ X, const T* __restrict__ spec,
                                                                     const T* __restrict__ tw, int n, int ss,
                                                                     int groups_per_rhs, int total_groups) {
  extern __shared__ unsigned char lds_raw[];
  T* buf = reinterpret_cast<T*>(lds_raw);
  const int tid = threadIdx.x;
  int c0;
  T* Xb = cols_reg_base<T, LOGN, H>(X, xcd_remap(blockIdx.x, total_groups), groups_per_rhs, total_groups, n, c0);
  T a[RegPlan<LOGN>::R0];
  cols_reg_load<T, LOGN, H>(Xb, a, tid, n);
  cols_reg_group<T, LOGN, H>(Xb, c0, a, buf, spec, tw, n, ss, tid);
}

// Column pass as two half-length problems (variants 6, 7).  A column has
// nonzeros only in its first N/2 entries, so its length-N transform splits
// into X[2k] = F_{N/2}(x)[k] and X[2k+1] = F_{N/2}(x_j W_N^j)[k]; after the
// spectrum multiply the kept outputs are y_j = F^-1(Y_even)[j] +
// W_N^-j F^-1(Y_odd)[j] (unnormalised inverses, j < N/2).  One workgroup
// (one wave for N <= 2048) per column, half the LDS of the full-length
// transform, and its barriers involve only that wave, so the waves of a CU
// run out of step: one loads while another transforms.  The even half's
// output stays in registers while the odd half runs.
template <int LOGN> struct EoPlan;
template <> struct EoPlan<10> { static constexpr int R0 = 8, R1 = 8, R2 = 8; };
template <> struct EoPlan<11> { static constexpr int R0 = 16, R1 = 16, R2 = 4; };
template <> struct EoPlan<12> { static constexpr int R0 = 16, R1 = 16, R2 = 8; };

template <typename T, int LOGN>
struct EoCfg {
  static constexpr int N = 1 << LOGN, M = N / 2;
  static constexpr int NT = M / EoPlan<LOGN>::R0;  // one first-pass butterfly per thread
  static constexpr int ROW = M + M / 16 + 2;
  static constexpr size_t lds() { return (size_t)ROW * sizeof(T); }
};

template <typename T, int LOGN, int H2>
__device__ __forceinline__ void eo_half(const T* __restrict__ Xb, T* a, T* buf, const T* __restrict__ spec,
                                        const T* __restrict__ tw, int n, int ss, int kxq, int tid) {
  using C = EoCfg<T, LOGN>;
  using PL = EoPlan<LOGN>;
  constexpr int N = C::N, M = C::M, ROW = C::ROW, NT = C::NT, W = Tile<T>::W;
  constexpr int R0 = PL::R0, R1 = PL::R1, R2 = PL::R2, NB0 = M / R0;
  // forward pass 0 from memory (odd half: times W_N^j, j = tid + r NB0, as
  // W_N^tid W_N^(r NB0): one per-lane table entry and R0 uniform ones)
  const T t0 = H2 ? tw[tid] : tmk<T>(1, 0);
#pragma unroll
  for (int r = 0; r < R0; ++r) {
    const int e = tid + r * NB0;
    T v = e < n ? Xb[(size_t)e * W] : tmk<T>(0, 0);
    if (H2 && r > 0) v = tmul(v, tw[r * NB0]);
    if (H2) v = tmul(v, t0);
    a[r] = v;
  }
  dft_r<T, R0, false>(a);
#pragma unroll
  for (int r = 0; r < R0; ++r) buf[lpad(tid * R0 + r)] = a[r];
  __syncthreads();
  reg_pass<T, M, R1, R0, 1, ROW, NT, false, N>(buf, tw, tid);
  {  // forward last pass, spectrum at ky = 2 k + H2, inverse first pass
    constexpr int NB = M / R2, NS = R0 * R1, PER = NB / NT;
    T b[PER][R2];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int j = tid + NT * q;
#pragma unroll
      for (int r = 0; r < R2; ++r) b[q][r] = buf[lpad(j + r * NB)];
    }
    __syncthreads();
  #pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int j = tid + NT * q;
      twiddle_r<T, N, R2, NS, false>(b[q], j, tw);
      dft_r<T, R2, false>(b[q]);
#pragma unroll
      for (int r = 0; r < R2; ++r) {
        const int ky = 2 * (j + r * NB) + H2;
        const int kyq = ky <= N / 2 ? ky : N - ky;
        b[q][r] = tmul(b[q][r], spec[(size_t)kxq * ss + kyq]);
      }
      dft_r<T, R2, true>(b[q]);
#pragma unroll
      for (int r = 0; r < R2; ++r) buf[lpad(j * R2 + r)] = b[q][r];
    }
  }
  __syncthreads();
  reg_pass<T, M, R1, R2, 1, ROW, NT, true, N>(buf, tw, tid);
  {  // inverse last pass: natural order, element tid + r NB0 in a[r]
    constexpr int NS = R2 * R1;
#pragma unroll
    for (int r = 0; r < R0; ++r) a[r] = buf[lpad(tid + r * NB0)];
    twiddle_r<T, N, R0, NS, true>(a, tid, tw);
    dft_r<T, R0, true>(a);
  }
}

template <typename T, int LOGN>
__global__ __launch_bounds__((EoCfg<T, LOGN>::NT)) void k_cols_eo(T* __restrict__ X, const T* __restrict__ spec,
                                                                const T* __restrict__ tw, int n, int ss,
                                                                int cols_per_rhs, int total) {
  using C = EoCfg<T, LOGN>;
  constexpr int N = C::N, W = Tile<T>::W, R0 = EoPlan<LOGN>::R0, NB0 = C::M / R0;
  extern __shared__ unsigned char lds_raw[];
  T* buf = reinterpret_cast<T*>(lds_raw);
  const int tid = threadIdx.x;
  const int g = xcd_remap(blockIdx.x, total);
  int b, c;
  col_group(g, cols_per_rhs, total, W, b, c);
  T* Xb = X + (size_t)b * n * N + (size_t)(c / W) * n * W + (c % W);
  const int kxq = c <= N / 2 ? c : N - c;
  T e[R0], o[R0];
  eo_half<T, LOGN, 0>(Xb, e, buf, spec, tw, n, ss, kxq, tid);
  __syncthreads();  // the even half's last reads before the odd half's first writes
  eo_half<T, LOGN, 1>(Xb, o, buf, spec, tw, n, ss, kxq, tid);
  T t0 = tw[tid];
  t0.y = -t0.y;
#pragma unroll
  for (int r = 0; r < R0; ++r) {
    const int j = tid + r * NB0;
    if (j < n) {
      T v = tmul(o[r], t0);
      if (r > 0) {
        T w = tw[r * NB0];
        w.y = -w.y;
        v = tmul(v, w);
      }
      Xb[(size_t)j * W] = tadd(e[r], v);
    }
  }
}

// Column pass with radix-8/4 register passes (variant 5): twice the threads
// per column of the radix-16 kernel (N/8 per column), so twice the waves
// in flight for the same LDS, at the cost of one more LDS exchange per
// transform.  Forward radices R0 R1 R2 R3, inverse R3 R2 R1 R0.
template <int LOGN> struct Reg4Plan;
template <> struct Reg4Plan<10> { static constexpr int R0 = 8, R1 = 8, R2 = 4, R3 = 4; };
template <> struct Reg4Plan<11> { static constexpr int R0 = 8, R1 = 8, R2 = 8, R3 = 4; };
template <> struct Reg4Plan<12> { static constexpr int R0 = 8, R1 = 8, R2 = 8, R3 = 8; };

template <typename T, int LOGN>
struct Reg4Cfg {
  static constexpr int N = 1 << LOGN;
  static constexpr int ROW = N + N / 16 + 2;  // as RegCfg
  // FP64 workgroups stay at 512 threads (more would cap registers at 128)
  static constexpr int MAXT = sizeof(T) == 16 ? 512 : 1024;
  static constexpr int fit(int c) {
    return (c * 2 * ROW * (int)sizeof(T) <= 153600 && c * 2 * N / 8 <= MAXT) ? fit(2 * c) : c;
  }
  static constexpr int CPW = fit(1) < Tile<T>::W ? fit(1) : Tile<T>::W;
  static constexpr int NT = CPW * N / 8;  // one radix-8 butterfly per thread
  static_assert(CPW <= Tile<T>::W, "a column group stays inside one tile");
  static constexpr size_t lds() { return (size_t)CPW * ROW * sizeof(T); }
};

template <typename T, int LOGN>
__global__ __launch_bounds__((Reg4Cfg<T, LOGN>::NT)) void k_cols_reg4(T* __restrict__ X, const T* __restrict__ spec,
                                                                     const T* __restrict__ tw, int n, int ss,
                                                                     int groups_per_rhs, int total_groups) {
  using C = Reg4Cfg<T, LOGN>;
  using PL = Reg4Plan<LOGN>;
  constexpr int N = C::N, CPW = C::CPW, ROW = C::ROW, W = Tile<T>::W, NT = C::NT;
  constexpr int R0 = PL::R0, R1 = PL::R1, R2 = PL::R2, R3 = PL::R3;
  extern __shared__ unsigned char lds_raw[];
  T* buf = reinterpret_cast<T*>(lds_raw);
  const int tid = threadIdx.x;
  const int g = xcd_remap(blockIdx.x, total_groups);
  int b, cg;
  col_group(g, groups_per_rhs, total_groups, W / CPW, b, cg);
  const int c0 = cg * CPW;
  T* Xb = X + (size_t)b * n * N + (size_t)(c0 / W) * n * W + (c0 % W);
  {  // forward pass 0 (radix R0, span 1) from memory, pruned input
    constexpr int NB = N / R0;
    int cc, j;
    bsplit<CPW>(tid, cc, j);
    T a[R0];
#pragma unroll
    for (int r = 0; r < R0; ++r) {
      const int e = j + r * NB;
      a[r] = e < n ? Xb[(size_t)e * W + cc] : tmk<T>(0, 0);
    }
    dft_r<T, R0, false>(a);
#pragma unroll
    for (int r = 0; r < R0; ++r) buf[cc * ROW + lpad(j * R0 + r)] = a[r];
  }
  __syncthreads();
  reg_pass<T, N, R1, R0, CPW, ROW, NT, false>(buf, tw, tid);
  reg_pass<T, N, R2, R0 * R1, CPW, ROW, NT, false>(buf, tw, tid);
  {  // forward last pass, spectrum, inverse first pass in registers
    constexpr int NB = N / R3, NS = R0 * R1 * R2, PER = CPW * NB / NT;
    T a[PER][R3];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int bi = tid + NT * q, cc = bi / NB, j = bi % NB;  // butterflies fastest (LDS, spectrum)
#pragma unroll
      for (int r = 0; r < R3; ++r) a[q][r] = buf[cc * ROW + lpad(j + r * NB)];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int bi = tid + NT * q, cc = bi / NB, j = bi % NB;  // butterflies fastest (LDS, spectrum)
      twiddle_r<T, N, R3, NS, false>(a[q], j, tw);
      dft_r<T, R3, false>(a[q]);
      const int kx = c0 + cc;
      const int kxq = kx <= N / 2 ? kx : N - kx;
#pragma unroll
      for (int r = 0; r < R3; ++r) {
        const int ky = j + r * NB;
        const int kyq = ky <= N / 2 ? ky : N - ky;
        a[q][r] = tmul(a[q][r], spec[(size_t)kxq * ss + kyq]);
      }
      dft_r<T, R3, true>(a[q]);
#pragma unroll
      for (int r = 0; r < R3; ++r) buf[cc * ROW + lpad(j * R3 + r)] = a[q][r];
    }
  }
  __syncthreads();
  reg_pass<T, N, R2, R3, CPW, ROW, NT, true>(buf, tw, tid);
  reg_pass<T, N, R1, R3 * R2, CPW, ROW, NT, true>(buf, tw, tid);
  {  // inverse last pass (radix R0): natural order, n kept outputs
    constexpr int NB = N / R0, NS = R3 * R2 * R1;
    int cc, j;
    bsplit<CPW>(tid, cc, j);
    T a[R0];
#pragma unroll
    for (int r = 0; r < R0; ++r) a[r] = buf[cc * ROW + lpad(j + r * NB)];
    twiddle_r<T, N, R0, NS, true>(a, j, tw);
    dft_r<T, R0, true>(a);
#pragma unroll
    for (int r = 0; r < R0; ++r) {
      const int e = j + r * NB;
      if (e < n) Xb[(size_t)e * W + cc] = a[r];
    }
  }
}

// K1 / K3 with the same register passes: CPW rows per workgroup; the first
// and last passes touch global memory with consecutive lanes on
// consecutive elements of a row (the middle pass only touches LDS).
template <int NB>
__device__ __forceinline__ void rsplit(int bi, int& cc, int& j) {
  cc = bi / NB;
  j = bi % NB;
}

template <typename T, typename R, int LOGN, int H>
__global__ __launch_bounds__((RegCfg<T, LOGN, H>::NT)) void k_rows_fwd_reg(const T* __restrict__ v,
                                                                          const R* __restrict__ m,
                                                                          T* __restrict__ X,
                                                                          const T* __restrict__ tw, int n,
                                                                          int total_rows) {
  using C = RegCfg<T, LOGN, H>;
  using PL = RegPlan<LOGN>;
  constexpr int N = C::N, CPW = C::CPW, ROW = C::ROW, NT = C::NT;
  constexpr int R0 = PL::R0, R1 = PL::R1, R2 = PL::R2;
  extern __shared__ unsigned char lds_raw[];
  T* buf = reinterpret_cast<T*>(lds_raw);
  const int tid = threadIdx.x;
  const int row0 = blockIdx.x * CPW;
  {  // pass 0 (radix 16, span 1) from memory: pad(m . v), n nonzero inputs
    constexpr int NB = N / R0;
    int cc, j;
    rsplit<NB>(tid, cc, j);
    const int row = row0 + cc;
    const bool live = row < total_rows;
    const int jr = live ? row % n : 0;
    T a[R0];
#pragma unroll
    for (int r = 0; r < R0; ++r) {
      const int i = j + r * NB;
      a[r] = tmk<T>(0, 0);
      if (live && i < n) {
        const T vv = v[(size_t)row * n + i];
        const R mm = m[(size_t)jr * n + i];
        a[r].x = vv.x * mm;
        a[r].y = vv.y * mm;
      }
    }
    dft_r<T, R0, false>(a);
#pragma unroll
    for (int r = 0; r < R0; ++r) buf[cc * ROW + lpad(j * R0 + r)] = a[r];
  }
  __syncthreads();
  reg_pass<T, N, R1, R0, CPW, ROW, NT, false>(buf, tw, tid);
  {  // last pass: natural order straight to the tiled intermediate
    constexpr int NB = N / R2, NS = R0 * R1, PER = CPW * NB / NT;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      int cc, j;
      rsplit<NB>(tid + NT * q, cc, j);
      T a[R2];
#pragma unroll
      for (int r = 0; r < R2; ++r) a[r] = buf[cc * ROW + lpad(j + r * NB)];
      twiddle_r<T, N, R2, NS, false>(a, j, tw);
      dft_r<T, R2, false>(a);
      const int row = row0 + cc;
      if (row < total_rows) {
#pragma unroll
        for (int r = 0; r < R2; ++r) X[tiled<T>(row / n, n, N, row % n, j + r * NB)] = a[r];
      }
    }
  }
}

template <typename T, int LOGN, int H>
__global__ __launch_bounds__((RegCfg<T, LOGN, H>::NT)) void k_rows_inv_reg(const T* __restrict__ X,
                                                                          const T* v, T* y,
                                                                          const T* __restrict__ tw, int n,
                                                                          int total_rows, double a_s,
                                                                          double b_s) {
  using C = RegCfg<T, LOGN, H>;
  using PL = RegPlan<LOGN>;
  constexpr int N = C::N, CPW = C::CPW, ROW = C::ROW, NT = C::NT;
  constexpr int R0 = PL::R0, R1 = PL::R1, R2 = PL::R2;
  extern __shared__ unsigned char lds_raw[];
  T* buf = reinterpret_cast<T*>(lds_raw);
  const int tid = threadIdx.x;
  const int row0 = blockIdx.x * CPW;
  {  // pass 0 from the tiled intermediate
    constexpr int NB = N / R0;
    int cc, j;
    rsplit<NB>(tid, cc, j);
    const int row = row0 + cc;
    T a[R0];
#pragma unroll
    for (int r = 0; r < R0; ++r)
      a[r] = row < total_rows ? X[tiled<T>(row / n, n, N, row % n, j + r * NB)] : tmk<T>(0, 0);
    dft_r<T, R0, true>(a);
#pragma unroll
    for (int r = 0; r < R0; ++r) buf[cc * ROW + lpad(j * R0 + r)] = a[r];
  }
  __syncthreads();
  reg_pass<T, N, R1, R0, CPW, ROW, NT, true>(buf, tw, tid);
  {  // last pass: natural order, the n kept outputs, y = a v + b conv
    constexpr int NB = N / R2, NS = R0 * R1, PER = CPW * NB / NT;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      int cc, j;
      rsplit<NB>(tid + NT * q, cc, j);
      T a[R2];
#pragma unroll
      for (int r = 0; r < R2; ++r) a[r] = buf[cc * ROW + lpad(j + r * NB)];
      twiddle_r<T, N, R2, NS, true>(a, j, tw);
      dft_r<T, R2, true>(a);
      const int row = row0 + cc;
      if (row >= total_rows) continue;
#pragma unroll
      for (int r = 0; r < R2; ++r) {
        const int i = j + r * NB;
        if (i >= n) continue;
        const size_t idx = (size_t)row * n + i;
        T conv = a[r];
        conv.x *= b_s;
        conv.y *= b_s;
        if (a_s != 0.0) {
          const T vv = v[idx];
          conv.x = fma((decltype(conv.x))a_s, vv.x, conv.x);
          conv.y = fma((decltype(conv.y))a_s, vv.y, conv.y);
        }
        y[idx] = conv;
      }
    }
  }
}

// K1 / K3 for FP64 rows with every LDS exchange made in two halves, real
// parts then imaginary parts: a row then needs one real per element of LDS
// (half the complex buffer), so the LDS limit on resident rows per CU (two
// waves per SIMD for FP64 at 2048 points) moves up to what registers allow
// (three for K1, four for K3), at twice the barriers per exchange.  Same
// passes, twiddles and arithmetic order as k_rows_fwd_reg / k_rows_inv_reg,
// so the results are the same bit for bit (FP32 rows keep the complex
// exchange: their LDS already allows what their registers do).

// a[PO][RO] to element positions po(q, r), then b[PI][RI] from positions
// pi(q, r), through the real buffer bx (real parts, then imaginary parts).
template <typename T, int PO, int RO, int PI, int RI, class FO, class FI>
__device__ __forceinline__ void xchg_halves(typename CT<T>::R* bx, const T (&a)[PO][RO], T (&b)[PI][RI], FO po,
                                            FI pi) {
#pragma unroll
  for (int q = 0; q < PO; ++q)
#pragma unroll
    for (int r = 0; r < RO; ++r) bx[po(q, r)] = a[q][r].x;
  __syncthreads();
#pragma unroll
  for (int q = 0; q < PI; ++q)
#pragma unroll
    for (int r = 0; r < RI; ++r) b[q][r].x = bx[pi(q, r)];
  __syncthreads();
#pragma unroll
  for (int q = 0; q < PO; ++q)
#pragma unroll
    for (int r = 0; r < RO; ++r) bx[po(q, r)] = a[q][r].y;
  __syncthreads();
#pragma unroll
  for (int q = 0; q < PI; ++q)
#pragma unroll
    for (int r = 0; r < RI; ++r) b[q][r].y = bx[pi(q, r)];
  __syncthreads();
}

template <typename T, int LOGN, int H>
struct SxCfg {
  using C = RegCfg<T, LOGN, H>;
  static constexpr size_t lds() { return (size_t)C::CPW * C::ROW * sizeof(typename CT<T>::R); }
};

// The middle pass of the row kernels on registers: butterflies bi = tid +
// NT q (q < P), radix R, span NS; returns nothing, a is transformed in place.
template <typename T, int N, int R, int NS, int P, int NT, bool INV>
__device__ __forceinline__ void mid_pass(T (&a)[P][R], const T* __restrict__ tw, int tid) {
  constexpr int NB = N / R;
#pragma unroll
  for (int q = 0; q < P; ++q) {
    const int j = (tid + NT * q) % NB;
    twiddle_r<T, N, R, NS, INV>(a[q], j, tw);
    dft_r<T, R, INV>(a[q]);
  }
}

template <typename T, typename R, int LOGN, int H>
__global__ __launch_bounds__((RegCfg<T, LOGN, H>::NT)) void k_rows_fwd_sx(const T* __restrict__ v,
                                                                         const R* __restrict__ m,
                                                                         T* __restrict__ X,
                                                                         const T* __restrict__ tw, int n,
                                                                         int total_rows) {
  using C = RegCfg<T, LOGN, H>;
  using PL = RegPlan<LOGN>;
  constexpr int N = C::N, CPW = C::CPW, ROW = C::ROW, NT = C::NT;
  constexpr int R0 = PL::R0, R1 = PL::R1, R2 = PL::R2;
  constexpr int NB0 = N / R0, NB1 = N / R1, NB2 = N / R2;
  constexpr int P1 = CPW * NB1 / NT, P2 = CPW * NB2 / NT;
  extern __shared__ unsigned char lds_raw[];
  typename CT<T>::R* bx = reinterpret_cast<typename CT<T>::R*>(lds_raw);
  const int tid = threadIdx.x;
  const int row0 = blockIdx.x * CPW;
  T a0[1][R0];
  int cc0, j0;
  rsplit<NB0>(tid, cc0, j0);
  {  // pass 0 (radix 16, span 1) from memory: pad(m . v), n nonzero inputs
    const int row = row0 + cc0;
    const bool live = row < total_rows;
    const int jr = live ? row % n : 0;
#pragma unroll
    for (int r = 0; r < R0; ++r) {
      const int i = j0 + r * NB0;
      a0[0][r] = tmk<T>(0, 0);
      if (live && i < n) {
        const T vv = v[(size_t)row * n + i];
        const R mm = m[(size_t)jr * n + i];
        a0[0][r].x = vv.x * mm;
        a0[0][r].y = vv.y * mm;
      }
    }
    dft_r<T, R0, false>(a0[0]);
  }
  T a1[P1][R1];
  xchg_halves<T, 1, R0, P1, R1>(
      bx, a0, a1, [&](int, int r) { return cc0 * ROW + lpad(j0 * R0 + r); },
      [&](int q, int r) {
        const int bi = tid + NT * q;
        return (bi / NB1) * ROW + lpad(bi % NB1 + r * NB1);
      });
  mid_pass<T, N, R1, R0, P1, NT, false>(a1, tw, tid);
  T a2[P2][R2];
  xchg_halves<T, P1, R1, P2, R2>(
      bx, a1, a2,
      [&](int q, int r) {
        const int bi = tid + NT * q, j = bi % NB1, k = j & (R0 - 1);
        return (bi / NB1) * ROW + lpad((j - k) * R1 + k + r * R0);
      },
      [&](int q, int r) {
        const int bi = tid + NT * q;
        return (bi / NB2) * ROW + lpad(bi % NB2 + r * NB2);
      });
  // last pass: natural order straight to the tiled intermediate
#pragma unroll
  for (int q = 0; q < P2; ++q) {
    int cc, j;
    rsplit<NB2>(tid + NT * q, cc, j);
    twiddle_r<T, N, R2, R0 * R1, false>(a2[q], j, tw);
    dft_r<T, R2, false>(a2[q]);
    const int row = row0 + cc;
    if (row < total_rows) {
#pragma unroll
      for (int r = 0; r < R2; ++r) X[tiled<T>(row / n, n, N, row % n, j + r * NB2)] = a2[q][r];
    }
  }
}

template <typename T, int LOGN, int H>
__global__ __launch_bounds__((RegCfg<T, LOGN, H>::NT)) void k_rows_inv_sx(const T* __restrict__ X,
                                                                         const T* v, T* y,
                                                                         const T* __restrict__ tw, int n,
                                                                         int total_rows, double a_s,
                                                                         double b_s) {
  using C = RegCfg<T, LOGN, H>;
  using PL = RegPlan<LOGN>;
  constexpr int N = C::N, CPW = C::CPW, ROW = C::ROW, NT = C::NT;
  constexpr int R0 = PL::R0, R1 = PL::R1, R2 = PL::R2;
  constexpr int NB0 = N / R0, NB1 = N / R1, NB2 = N / R2;
  constexpr int P1 = CPW * NB1 / NT, P2 = CPW * NB2 / NT;
  extern __shared__ unsigned char lds_raw[];
  typename CT<T>::R* bx = reinterpret_cast<typename CT<T>::R*>(lds_raw);
  const int tid = threadIdx.x;
  const int row0 = blockIdx.x * CPW;
  T a0[1][R0];
  int cc0, j0;
  rsplit<NB0>(tid, cc0, j0);
  {  // pass 0 from the tiled intermediate
    const int row = row0 + cc0;
#pragma unroll
    for (int r = 0; r < R0; ++r)
      a0[0][r] = row < total_rows ? X[tiled<T>(row / n, n, N, row % n, j0 + r * NB0)] : tmk<T>(0, 0);
    dft_r<T, R0, true>(a0[0]);
  }
  T a1[P1][R1];
  xchg_halves<T, 1, R0, P1, R1>(
      bx, a0, a1, [&](int, int r) { return cc0 * ROW + lpad(j0 * R0 + r); },
      [&](int q, int r) {
        const int bi = tid + NT * q;
        return (bi / NB1) * ROW + lpad(bi % NB1 + r * NB1);
      });
  mid_pass<T, N, R1, R0, P1, NT, true>(a1, tw, tid);
  T a2[P2][R2];
  xchg_halves<T, P1, R1, P2, R2>(
      bx, a1, a2,
      [&](int q, int r) {
        const int bi = tid + NT * q, j = bi % NB1, k = j & (R0 - 1);
        return (bi / NB1) * ROW + lpad((j - k) * R1 + k + r * R0);
      },
      [&](int q, int r) {
        const int bi = tid + NT * q;
        return (bi / NB2) * ROW + lpad(bi % NB2 + r * NB2);
      });
  // last pass: natural order, the n kept outputs, y = a v + b conv
#pragma unroll
  for (int q = 0; q < P2; ++q) {
    int cc, j;
    rsplit<NB2>(tid + NT * q, cc, j);
    twiddle_r<T, N, R2, R0 * R1, true>(a2[q], j, tw);
    dft_r<T, R2, true>(a2[q]);
    const int row = row0 + cc;
    if (row >= total_rows) continue;
#pragma unroll
    for (int r = 0; r < R2; ++r) {
      const int i = j + r * NB2;
      if (i >= n) continue;
      const size_t idx = (size_t)row * n + i;
      T conv = a2[q][r];
      conv.x *= b_s;
      conv.y *= b_s;
      if (a_s != 0.0) {
        const T vv = v[idx];
        conv.x = fma((decltype(conv.x))a_s, vv.x, conv.x);
        conv.y = fma((decltype(conv.y))a_s, vv.y, conv.y);
      }
      y[idx] = conv;
    }
  }
}

// K3: y = a v + b * (first n of IFFT_rows(X)).
template <typename T, int LOGN>
__global__ __launch_bounds__(RowCfg<LOGN>::NT) void k_rows_inv(const T* __restrict__ X,
                                                             const T* v, T* y,
                                                             const T* __restrict__ tw, int n,
                                                             int total_rows, double a, double bsc) {
  using C = RowCfg<LOGN>;
  constexpr int N = C::N;
  extern __shared__ unsigned char lds_raw[];
  T* buf = reinterpret_cast<T*>(lds_raw);
  const int tid = threadIdx.x;
  const int row0 = blockIdx.x * C::COUNT;
  for (int e = tid; e < C::COUNT * N; e += C::NT) {
    const int c = e / N, kx = e % N;
    const int row = row0 + c;
    T val = tmk<T>(0, 0);
    if (row < total_rows) val = X[tiled<T>(row / n, n, N, row % n, kx)];
    buf[e] = val;
  }
  __syncthreads();
  fft_lds<T, LOGN, C::COUNT, N, C::NT, true>(buf, tw, tid);
  for (int e = tid; e < C::COUNT * n; e += C::NT) {
    const int c = e / n, i = e % n;
    const int row = row0 + c;
    if (row < total_rows) {
      const size_t idx = (size_t)row * n + i;
      T conv = buf[c * N + i];
      conv.x *= bsc;
      conv.y *= bsc;
      if (a != 0.0) {
        const T vv = v[idx];
        conv.x = fma((decltype(conv.x))a, vv.x, conv.x);
        conv.y = fma((decltype(conv.y))a, vv.y, conv.y);
      }
      y[idx] = conv;
    }
  }
}

// Setup: forward FFT of every row of a P x P row-major array, in place.
template <int LOGN>
__global__ __launch_bounds__(RowCfg<LOGN>::NT) void k_full_rows(cplx* __restrict__ c,
                                                              const cplx* __restrict__ tw) {
  using C = RowCfg<LOGN>;
  constexpr int N = C::N;
  extern __shared__ unsigned char lds_raw[];
  cplx* buf = reinterpret_cast<cplx*>(lds_raw);
  const int tid = threadIdx.x;
  const int row0 = blockIdx.x * C::COUNT;
  for (int e = tid; e < C::COUNT * N; e += C::NT)
    buf[e] = (row0 + e / N < N) ? c[(size_t)row0 * N + e] : cmk(0.0, 0.0);
  __syncthreads();
  fft_lds<cplx, LOGN, C::COUNT, N, C::NT, false>(buf, tw, tid);
  for (int e = tid; e < C::COUNT * N; e += C::NT)
    if (row0 + e / N < N) c[(size_t)row0 * N + e] = buf[e];
}

// Setup: forward FFT of every column, in place.
template <int LOGN>
__global__ __launch_bounds__((ColCfg<cplx, LOGN, 0>::NT)) void k_full_cols(cplx* __restrict__ c,
                                                                       const cplx* __restrict__ tw) {
  using C = ColCfg<cplx, LOGN, 0>;
  constexpr int N = C::N, CPW = C::CPW, S = C::STRIDE;
  extern __shared__ unsigned char lds_raw[];
  cplx* buf = reinterpret_cast<cplx*>(lds_raw);
  const int tid = threadIdx.x;
  const int c0 = blockIdx.x * CPW;
  for (int e = tid; e < CPW * N; e += C::NT) {
    const int j = e / CPW, cc = e % CPW;
    buf[cc * S + j] = c[(size_t)j * N + c0 + cc];
  }
  __syncthreads();
  fft_lds<cplx, LOGN, CPW, S, C::NT, false>(buf, tw, tid);
  for (int e = tid; e < CPW * N; e += C::NT) {
    const int j = e / CPW, cc = e % CPW;
    c[(size_t)j * N + c0 + cc] = buf[cc * S + j];
  }
}

template <typename T>
__global__ void k_extract_quarter(const cplx* __restrict__ c, T* __restrict__ spec, int P,
                                  double scale) {
  const int ss = P / 2 + 1;
  const int kx = blockIdx.x * blockDim.x + threadIdx.x;
  const int ky = blockIdx.y;
  if (kx >= ss) return;
  const cplx v = c[(size_t)ky * P + kx];
  spec[(size_t)ky * ss + kx] = tmk<T>(v.x * scale, v.y * scale);
}

template <typename K>
hipError_t set_lds(K kernel, size_t bytes) {
  if (bytes <= 65536) return hipSuccess;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

// Raises a kernel's dynamic-LDS limit once per process (function-local
// statics initialise once even when several host threads launch: the
// many-plan entry points drive plans from one thread each).
#define LS_SET_LDS_ONCE(...)                                    \
  do {                                                          \
    static const hipError_t once_ = set_lds(__VA_ARGS__);       \
    LS_HIP(once_);                                              \
  } while (0)

template <typename T, int LOGN, int V>
ls_status run_cols(const ApplyView<T, typename CT<T>::R>& av, int batch) {
  using CC = ColCfg<T, LOGN, V>;
  constexpr int N = 1 << LOGN;
  const size_t lds_c = (size_t)CC::CPW * CC::STRIDE * sizeof(T);
  LS_SET_LDS_ONCE((k_cols_conv<T, LOGN, V>), lds_c);
  const int gpr = N / CC::CPW;
  const int groups = gpr * batch;
  k_cols_conv<T, LOGN, V><<<groups, CC::NT, lds_c, av.stream>>>(av.work, av.spec, av.tw, av.n,
                                                               av.ss, gpr, groups);
  LS_HIP(hipGetLastError());
  return LS_OK;
}

template <typename T, int LOGN, int H>
ls_status run_cols_reg(const ApplyView<T, typename CT<T>::R>& av, int batch) {
  using RC = RegCfg<T, LOGN, H>;
  constexpr int N = 1 << LOGN;
  LS_SET_LDS_ONCE((k_cols_reg<T, LOGN, H>), RC::lds());
  const int gpr = N / RC::CPW;
  const int groups = gpr * batch;
  k_cols_reg<T, LOGN, H><<<groups, RC::NT, RC::lds(), av.stream>>>(av.work, av.spec, av.tw, av.n, av.ss,
                                                                    gpr, groups);
  LS_HIP(hipGetLastError());
  return LS_OK;
}

template <typename T, int LOGN>
ls_status run_cols_eo(const ApplyView<T, typename CT<T>::R>& av, int batch) {
  using C = EoCfg<T, LOGN>;
  constexpr int N = 1 << LOGN;
  LS_SET_LDS_ONCE((k_cols_eo<T, LOGN>), C::lds());
  const int total = N * batch;
  k_cols_eo<T, LOGN><<<total, C::NT, C::lds(), av.stream>>>(av.work, av.spec, av.tw, av.n, av.ss, N, total);
  LS_HIP(hipGetLastError());
  return LS_OK;
}

template <typename T, int LOGN>
ls_status run_cols_reg4(const ApplyView<T, typename CT<T>::R>& av, int batch) {
  using RC = Reg4Cfg<T, LOGN>;
  constexpr int N = 1 << LOGN;
  LS_SET_LDS_ONCE((k_cols_reg4<T, LOGN>), RC::lds());
  const int gpr = N / RC::CPW;
  const int groups = gpr * batch;
  k_cols_reg4<T, LOGN><<<groups, RC::NT, RC::lds(), av.stream>>>(av.work, av.spec, av.tw, av.n, av.ss, gpr,
                                                                  groups);
  LS_HIP(hipGetLastError());
  return LS_OK;
}

template <typename T, typename R, int LOGN>
ls_status run_apply(const ApplyView<T, R>& av, const T* v, T* y, int batch, double a, double b) {
  using RC = RowCfg<LOGN>;
  constexpr int N = 1 << LOGN;
  const int n = av.n;
  const int rows = batch * n;
  const size_t lds_r = (size_t)RC::COUNT * N * sizeof(T);
  LS_SET_LDS_ONCE((k_rows_fwd<T, R, LOGN>), lds_r);
  LS_SET_LDS_ONCE((k_rows_inv<T, LOGN>), lds_r);
  constexpr bool reg = LOGN >= 10 && LOGN <= 12;
  using RR = RegCfg<T, LOGN, kRowHalf>;
  constexpr bool sx = reg && std::is_same<T, cplx>::value;
  using SX = SxCfg<T, LOGN, kRowHalf>;
  if constexpr (sx) {
    LS_SET_LDS_ONCE((k_rows_fwd_sx<T, R, LOGN, kRowHalf>), SX::lds());
    LS_SET_LDS_ONCE((k_rows_inv_sx<T, LOGN, kRowHalf>), SX::lds());
    k_rows_fwd_sx<T, R, LOGN, kRowHalf><<<(rows + RR::CPW - 1) / RR::CPW, RR::NT, SX::lds(), av.stream>>>(
        v, av.m, av.work, av.tw, n, rows);
  } else if constexpr (reg) {
    LS_SET_LDS_ONCE((k_rows_fwd_reg<T, R, LOGN, kRowHalf>), RR::lds());
    LS_SET_LDS_ONCE((k_rows_inv_reg<T, LOGN, kRowHalf>), RR::lds());
    k_rows_fwd_reg<T, R, LOGN, kRowHalf><<<(rows + RR::CPW - 1) / RR::CPW, RR::NT, RR::lds(), av.stream>>>(
        v, av.m, av.work, av.tw, n, rows);
  } else {
    k_rows_fwd<T, R, LOGN><<<(rows + RC::COUNT - 1) / RC::COUNT, RC::NT, lds_r, av.stream>>>(
        v, av.m, av.work, av.tw, n, rows);
  }
  LS_HIP(hipGetLastError());
  switch (av.col_variant) {
    case 1:
      if constexpr (reg) LS_TRY((run_cols_reg<T, LOGN, 1>(av, batch)));
      else LS_TRY((run_cols<T, LOGN, 1>(av, batch)));
      break;
    case 2: LS_TRY((run_cols<T, LOGN, 0>(av, batch))); break;
    case 3: LS_TRY((run_cols<T, LOGN, 1>(av, batch))); break;
    case 4: LS_TRY((run_cols<T, LOGN, 2>(av, batch))); break;
    case 5:
      if constexpr (reg) LS_TRY((run_cols_reg4<T, LOGN>(av, batch)));
      else LS_TRY((run_cols<T, LOGN, 0>(av, batch)));
      break;
    case 6:
      if constexpr (reg) LS_TRY((run_cols_eo<T, LOGN>(av, batch)));
      else LS_TRY((run_cols<T, LOGN, 0>(av, batch)));
      break;
    case 7:
      if constexpr (reg) LS_TRY((run_cols_reg<T, LOGN, 2>(av, batch)));
      else LS_TRY((run_cols<T, LOGN, 2>(av, batch)));
      break;
    default:
      if constexpr (reg) LS_TRY((run_cols_reg<T, LOGN, 0>(av, batch)));
      else LS_TRY((run_cols<T, LOGN, 0>(av, batch)));
      break;
  }
  if constexpr (sx)
    k_rows_inv_sx<T, LOGN, kRowHalf><<<(rows + RR::CPW - 1) / RR::CPW, RR::NT, SX::lds(), av.stream>>>(
        av.work, v, y, av.tw, n, rows, a, b);
  else if constexpr (reg)
    k_rows_inv_reg<T, LOGN, kRowHalf><<<(rows + RR::CPW - 1) / RR::CPW, RR::NT, RR::lds(), av.stream>>>(
        av.work, v, y, av.tw, n, rows, a, b);
  else
    k_rows_inv<T, LOGN><<<(rows + RC::COUNT - 1) / RC::COUNT, RC::NT, lds_r, av.stream>>>(
        av.work, v, y, av.tw, n, rows, a, b);
  LS_HIP(hipGetLastError());
  return LS_OK;
}

template <int LOGN>
ls_status run_full_forward(ls_plan* p, cplx* c) {
  using RC = RowCfg<LOGN>;
  using CC = ColCfg<cplx, LOGN, 0>;
  constexpr int N = 1 << LOGN;
  const size_t lds_r = (size_t)RC::COUNT * N * sizeof(cplx);
  const size_t lds_c = (size_t)CC::CPW * CC::STRIDE * sizeof(cplx);
  LS_HIP(set_lds(k_full_rows<LOGN>, lds_r));
  LS_HIP(set_lds(k_full_cols<LOGN>, lds_c));
  k_full_rows<LOGN><<<(N + RC::COUNT - 1) / RC::COUNT, RC::NT, lds_r, p->stream>>>(c, p->tw);
  LS_HIP(hipGetLastError());
  k_full_cols<LOGN><<<N / CC::CPW, CC::NT, lds_c, p->stream>>>(c, p->tw);
  LS_HIP(hipGetLastError());
  return LS_OK;
}

}  // namespace

template <typename T>
static ls_status twiddles_to(ls_plan* p, T** dst) {
  const int P = p->P;
  std::vector<T> h(P);
  const long double twopi = 6.283185307179586476925286766559005768L;
  for (int k = 0; k < P; ++k) {
    const long double ang = -twopi * (long double)k / (long double)P;
    h[k] = tmk<T>((double)cosl(ang), (double)sinl(ang));
  }
  LS_TRY(plan_alloc(p, (void**)dst, sizeof(T) * P));
  LS_HIP(hipMemcpyAsync(*dst, h.data(), sizeof(T) * P, hipMemcpyHostToDevice, p->stream));
  LS_HIP(hipStreamSynchronize(p->stream));
  return LS_OK;
}

ls_status fft_setup_twiddles(ls_plan* p) {
  LS_TRY(twiddles_to<cplx>(p, &p->tw));
  if (p->fp32) LS_TRY(twiddles_to<fcplx>(p, &p->f32.tw));
  return LS_OK;
}

#define LS_DISPATCH_LOGP(LOGP, CALL)                 \
  switch (LOGP) {                                    \
    case 4: return CALL(4);                          \
    case 5: return CALL(5);                          \
    case 6: return CALL(6);                          \
    case 7: return CALL(7);                          \
    case 8: return CALL(8);                          \
    case 9: return CALL(9);                          \
    case 10: return CALL(10);                        \
    case 11: return CALL(11);                        \
    case 12: return CALL(12);                        \
    default:                                         \
      ls_set_error("unsupported FFT size");          \
      return LS_EUNSUPPORTED;                        \
  }

ls_status fft2_full_forward(ls_plan* p, cplx* c) {
#define CALL_FULL(L) run_full_forward<L>(p, c)
  LS_DISPATCH_LOGP(p->logP, CALL_FULL)
#undef CALL_FULL
}

__global__ void k_spec_to_f32(const cplx* __restrict__ a, fcplx* __restrict__ b, size_t cnt) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < cnt) b[i] = make_float2((float)a[i].x, (float)a[i].y);
}

// FP32 copy of the stored FP64 spectrum (the same rounding as extracting it
// from the transform in FP32).
ls_status spectrum_to_f32(ls_plan* p) {
  const size_t cnt = (size_t)p->spec_side * p->spec_side;
  k_spec_to_f32<<<(unsigned)((cnt + 255) / 256), 256, 0, p->stream>>>(p->spec, p->f32.spec, cnt);
  LS_HIP(hipGetLastError());
  return LS_OK;
}

ls_status spectrum_extract(ls_plan* p, const cplx* c) {
  const int ss = p->P / 2 + 1;
  const double scale = p->omega * p->omega / ((double)p->P * (double)p->P);
  dim3 grid((ss + 255) / 256, ss);
  k_extract_quarter<cplx><<<grid, 256, 0, p->stream>>>(c, p->spec, p->P, scale);
  if (p->fp32) k_extract_quarter<fcplx><<<grid, 256, 0, p->stream>>>(c, p->f32.spec, p->P, scale);
  LS_HIP(hipGetLastError());
  return LS_OK;
}

template <typename T, typename R>
ls_status apply_H_one(const ApplyView<T, R>& av, int logP, const T* v, T* y, int batch, double a, double b) {
#define CALL_APPLY(L) run_apply<T, R, L>(av, v, y, batch, a, b)
  LS_DISPATCH_LOGP(logP, CALL_APPLY)
#undef CALL_APPLY
}

// The batch runs in chunks whose n x P intermediate is at most 96 MB: it is
// written by the row pass and read back by the column and inverse row passes
// while still in the 256 MB Infinity Cache (measured at 1024^2, batch 8,
// FP64: 0.486 ms in one piece, 0.444 ms in chunks of 3; 64 and 128 MB caps
// 0.452 / 0.453 ms).
constexpr size_t kApplyChunkBytes = (size_t)96 << 20;

template <typename T, typename R>
ls_status apply_H_t(const ApplyView<T, R>& av, int logP, const T* v, T* y, int batch, double a,
                    double b) {
  const size_t inter = (size_t)av.n * ((size_t)1 << logP) * sizeof(T);
  const int chunk = std::max(1, (int)(kApplyChunkBytes / inter));
  const size_t N = (size_t)av.n * av.n;
  for (int b0 = 0; b0 < batch; b0 += chunk)
    LS_TRY((apply_H_one<T, R>(av, logP, v + b0 * N, y + b0 * N, std::min(chunk, batch - b0), a, b)));
  return LS_OK;
}

// y = a v + b (omega^2 G (m v)); a = 1, b = 1 gives H v; a = 0, b = -1 gives
// f = -omega^2 G (m u_I).
ls_status apply_H(ls_plan* p, const cplx* v, cplx* y, int batch, double a, double b) {
  return apply_H_t<cplx, double>(view64(p), p->logP, v, y, batch, a, b);
}

ls_status apply_H32(ls_plan* p, const fcplx* v, fcplx* y, int batch, double a, double b) {
  return apply_H_t<fcplx, float>(view32(p), p->logP, v, y, batch, a, b);
}

// FFT autotuner: times every column-pass variant on `batch` vectors of this
// plan with HIP events on the plan's stream and keeps the fastest, for the
// FP64 and (FP32 plans) FP32 operator.  Two rounds over all variants, each
// variant's better round counts, so that the order of the variants and the
// warm-up of caches do not decide.
template <typename T, typename R>
static ls_status tune_one(ls_plan* p, ApplyView<T, R> av, T* in, T* out, int batch, int* choice,
                          float* ms_out) {
  hipEvent_t e0, e1;
  LS_HIP(hipEventCreate(&e0));
  LS_HIP(hipEventCreate(&e1));
  for (int v = 0; v < kColVariants; ++v) ms_out[v] = 1e30f;
  for (int round = 0; round < 2; ++round) {
    for (int v = 0; v < kColVariants; ++v) {
      av.col_variant = v;
      LS_TRY((apply_H_t<T, R>(av, p->logP, in, out, batch, 1.0, 1.0)));
      LS_HIP(hipEventRecord(e0, p->stream));
      for (int r = 0; r < 3; ++r) LS_TRY((apply_H_t<T, R>(av, p->logP, in, out, batch, 1.0, 1.0)));
      LS_HIP(hipEventRecord(e1, p->stream));
      LS_HIP(hipEventSynchronize(e1));
      float ms = 0.f;
      LS_HIP(hipEventElapsedTime(&ms, e0, e1));
      ms_out[v] = std::min(ms_out[v], ms / 3.f);
    }
  }
  int arg = 0;
  for (int v = 1; v < kColVariants; ++v)
    if (ms_out[v] < ms_out[arg]) arg = v;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *choice = arg;
  return LS_OK;
}

ls_status fft_autotune(ls_plan* p) {
  const int batch = p->opt.max_batch;
  const size_t N = (size_t)p->n * p->n;
  // inputs: the plan's grid scratch (contents irrelevant for timing)
  LS_TRY(vec_zero(p, p->vtmp, N * batch));
  LS_TRY((tune_one<cplx, double>(p, view64(p), p->vtmp, p->vtmp + N * batch, batch,
                                  &p->col_variant64, p->tune_ms64)));
  if (p->fp32) {
    LS_TRY(vec_zero(p, p->vtmp32, N * batch));
    LS_TRY((tune_one<fcplx, float>(p, view32(p), p->vtmp32, p->vtmp32 + N * batch, batch,
                                   &p->col_variant32, p->tune_ms32)));
  }
  return LS_OK;
}
