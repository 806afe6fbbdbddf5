// Fourier-neural-operator preconditioner: bf16 MFMA products, the network's
// forward and backward passes, loss, Adam, and its use as a residual map.
//
// Every dense product of the network is one call of a strided, batched
// GEMM on gfx950 matrix cores (v_mfma_f32_16x16x32_bf16): operands are
// stored in FP32, rounded to bf16 when staged in LDS, and accumulated in
// FP32.  The truncated spectral transforms are products with small DFT
// matrices (n x 32, 64 x n), not FFTs: only 16 x 32 of the n^2 modes are
// kept, so the dense form does 32 multiply-adds per point and pass on
// matrix cores instead of a full-length FFT.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <map>

#include "../../include/ls_fno.h"
#include "ls_internal.h"

namespace {

constexpr int kW = LS_FNO_WIDTH, kM = LS_FNO_MODES, kL = LS_FNO_LAYERS, kH = LS_FNO_HIDDEN;
constexpr int kKZ = 2 * kM;  // retained kz values
constexpr int kIn = 5, kOut = 2;

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// GELU (erf form) and its derivative
__device__ __forceinline__ float gelu_f(float x) { return 0.5f * x * (1.f + erff(x * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_d(float x) {
  return 0.5f * (1.f + erff(x * 0.70710678118654752f)) + x * expf(-0.5f * x * x) * 0.39894228040143268f;
}

// ------------------------------------------------------------------ GEMM
struct GemmP {
  int M, N, K;
  const float* A;
  long long sam, sak, sab, sag;  // sag: offset per K segment
  const float* B;
  long long sbk, sbn, sbb, sbg;
  float* C;
  long long scm, scn, scb;
  int kseg;      // K segment length (multiple of 32), 0 = one segment
  int klen;      // K elements per split
  float alpha, beta;
  const float* bias_m;  // added to row m (split 0 only)
  int atomic;           // split K: accumulate with atomic adds
  float* C2;            // if set: GELU of the result, same layout as C (C may then be null)
  const __bf16* Ah;     // if set: A stored as bf16 (read in place of A)
};

// Tile BM x BN x 32, 256 threads = 4 waves in a WM x WN grid; each wave
// owns (BM/WM) x (BN/WN) outputs as 16 x 16 MFMA blocks.  Operands are
// staged k-contiguous in LDS (rows padded to 40 bf16 = 80 bytes, so the 16
// rows one 16-byte read touches fall in distinct banks).  The next K tile's
// global loads are issued before the current tile's MFMAs.
template <int BM, int BN, int WM, int WN, typename TA = float>
__global__ __launch_bounds__(256) void k_gemm_bf16(GemmP g) {
  constexpr int BK = 32, LDK = 40;
  constexpr int TM = BM / WM, TN = BN / WN, FM = TM / 16, FN = TN / 16;
  constexpr int EA = BM * BK / 256, EB = BN * BK / 256;
  static_assert(WM * WN == 4 && FM >= 1 && FN >= 1, "tile shape");
  __shared__ __attribute__((aligned(16))) __bf16 As[BM * LDK];
  __shared__ __attribute__((aligned(16))) __bf16 Bs[BN * LDK];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN;
  const int tilesN = (g.N + BN - 1) / BN;
  const int m0 = (blockIdx.x / tilesN) * BM, n0 = (blockIdx.x % tilesN) * BN;
  const long long b = blockIdx.y;
  const int kb = blockIdx.z * g.klen;
  const int ke = min(g.K, kb + g.klen);
  const TA* __restrict__ A;
  if constexpr (sizeof(TA) == 2) A = g.Ah + b * g.sab;
  else A = g.A + b * g.sab;
  const float* __restrict__ B = g.B + b * g.sbb;
  const bool akf = g.sak == 1, bkf = g.sbk == 1;
  float ra[EA], rb[EB];
  auto amap = [&](int e, int& m, int& k) {
    const int idx = tid + e * 256;
    if (akf) { m = idx / BK; k = idx % BK; } else { m = idx % BM; k = idx / BM; }
  };
  auto bmap = [&](int e, int& n, int& k) {
    const int idx = tid + e * 256;
    if (bkf) { n = idx / BK; k = idx % BK; } else { n = idx % BN; k = idx / BN; }
  };
  auto load = [&](int k0) {
    long long ao = 0, bo = 0;
    int kin = k0;
    if (g.kseg > 0) {
      const int sg = k0 / g.kseg;
      kin = k0 - sg * g.kseg;
      ao = sg * g.sag;
      bo = sg * g.sbg;
    }
#pragma unroll
    for (int e = 0; e < EA; ++e) {
      int m, k;
      amap(e, m, k);
      ra[e] = (m0 + m < g.M && k0 + k < ke) ? (float)A[ao + (m0 + m) * g.sam + (long long)(kin + k) * g.sak] : 0.f;
    }
#pragma unroll
    for (int e = 0; e < EB; ++e) {
      int n, k;
      bmap(e, n, k);
      rb[e] = (n0 + n < g.N && k0 + k < ke) ? B[bo + (long long)(kin + k) * g.sbk + (n0 + n) * g.sbn] : 0.f;
    }
  };
  f32x4 acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  if (kb < ke) load(kb);
  for (int k0 = kb; k0 < ke; k0 += BK) {
    __syncthreads();
#pragma unroll
    for (int e = 0; e < EA; ++e) {
      int m, k;
      amap(e, m, k);
      As[m * LDK + k] = (__bf16)ra[e];
    }
#pragma unroll
    for (int e = 0; e < EB; ++e) {
      int n, k;
      bmap(e, n, k);
      Bs[n * LDK + k] = (__bf16)rb[e];
    }
    __syncthreads();
    if (k0 + BK < ke) load(k0 + BK);
    const int r16 = lane & 15, kq = (lane >> 4) * 8;
#pragma unroll
    for (int i = 0; i < FM; ++i) {
      const bf16x8 av = *reinterpret_cast<const bf16x8*>(&As[(wm * TM + i * 16 + r16) * LDK + kq]);
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        const bf16x8 bv = *reinterpret_cast<const bf16x8*>(&Bs[(wn * TN + j * 16 + r16) * LDK + kq]);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc[i][j], 0, 0, 0);
      }
    }
  }
  // D layout: lane holds rows 4*(lane/16) + 0..3 of column lane % 16
  float* __restrict__ C = g.C ? g.C + b * g.scb : nullptr;
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int m = m0 + wm * TM + i * 16 + (lane >> 4) * 4 + t;
        const int n = n0 + wn * TN + j * 16 + (lane & 15);
        if (m >= g.M || n >= g.N) continue;
        float v = g.alpha * acc[i][j][t];
        if (g.bias_m && blockIdx.z == 0) v += g.bias_m[m];
        const long long co = b * g.scb + m * g.scm + n * g.scn;
        if (g.C2) {  // single split, beta = 0
          if (g.C) g.C[co] = v;
          g.C2[co] = gelu_f(v);
          continue;
        }
        float* c = C + m * g.scm + n * g.scn;
        if (g.atomic)
          atomicAdd(c, v);
        else
          *c = (g.beta != 0.f ? g.beta * *c : 0.f) + v;
      }
}

__global__ void k_fill_strided(float* C, int M, int N, long long scm, long long scn,
                               long long scb, float val) {
  const long long b = blockIdx.y;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < (long long)M * N;
       e += (long long)gridDim.x * blockDim.x) {
    const int m = (int)(e / N), n = (int)(e % N);
    C[b * scb + m * scm + n * scn] = val;
  }
}

__global__ void k_scale_strided(float* C, int M, int N, long long scm, long long scn,
                                long long scb, float s) {
  const long long b = blockIdx.y;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < (long long)M * N;
       e += (long long)gridDim.x * blockDim.x) {
    const int m = (int)(e / N), n = (int)(e % N);
    C[b * scb + m * scm + n * scn] *= s;
  }
}

template <int BM, int BN, int WM, int WN, typename TA = float>
void launch_gemm(const GemmP& g, int batch, int splits, hipStream_t st) {
  const int tiles = ((g.M + BM - 1) / BM) * ((g.N + BN - 1) / BN);
  k_gemm_bf16<BM, BN, WM, WN, TA><<<dim3(tiles, batch, splits), 256, 0, st>>>(g);
}

// Tile shape for an M x N output, split-K count for long reductions with
// few output tiles; every product of the network goes through here.
ls_status gemm(GemmP g, int batch, hipStream_t st) {
  if (g.M <= 0 || g.N <= 0 || batch <= 0) return LS_OK;
  if (g.kseg < 0 || (g.kseg > 0 && g.kseg % 32 != 0)) {
    ls_set_error("bf16 GEMM: K segment length must be a multiple of 32");
    return LS_EINVAL;
  }
  int bm, bn;
  if (g.M <= 16) { bm = 16; bn = 64; }
  else if (g.M <= 32) { bm = 32; bn = g.N <= 32 ? 32 : 128; }
  else if (g.N <= 16) { bm = 64; bn = 16; }
  else if (g.N <= 32) { bm = g.M >= 128 ? 128 : 64; bn = 32; }
  else { bm = 64; bn = 64; }
  const long long tiles = (long long)((g.M + bm - 1) / bm) * ((g.N + bn - 1) / bn) * batch;
  int splits = 1;
  if (g.K <= 0) {  // C = beta C (+ bias): one pass with no K tiles
    g.klen = 32;
    g.atomic = 0;
    if (bm == 16) launch_gemm<16, 64, 1, 4>(g, batch, 1, st);
    else launch_gemm<64, 64, 2, 2>(g, batch, 1, st);
    LS_HIP(hipGetLastError());
    return LS_OK;
  }
  if (g.C2 && g.beta != 0.f) {
    ls_set_error("bf16 GEMM: a GELU output needs beta = 0");
    return LS_EINVAL;
  }
  if (tiles < 512 && g.K >= 1024 && !g.C2) {
    splits = (int)std::min<long long>((1024 + tiles - 1) / tiles, g.K / 512);
    if (splits < 1) splits = 1;
  }
  g.klen = ((g.K + splits - 1) / splits + 31) / 32 * 32;
  splits = (g.K + g.klen - 1) / g.klen;
  g.atomic = splits > 1;
  if (g.atomic) {
    // the splits add into C: prepare beta * C first
    const int blocks = (int)std::min<long long>(1024, ((long long)g.M * g.N + 255) / 256);
    if (g.beta == 0.f)
      k_fill_strided<<<dim3(blocks, batch), 256, 0, st>>>(g.C, g.M, g.N, g.scm, g.scn, g.scb, 0.f);
    else if (g.beta != 1.f)
      k_scale_strided<<<dim3(blocks, batch), 256, 0, st>>>(g.C, g.M, g.N, g.scm, g.scn, g.scb, g.beta);
  }
  if (g.Ah) {  // bf16 activations (inference): the x-transform shape only
    if (bm != 128 || bn != 32) {
      ls_set_error("bf16 GEMM: a bf16 A operand is supported for M >= 128, N = 32 only");
      return LS_EINVAL;
    }
    launch_gemm<128, 32, 4, 1, __bf16>(g, batch, splits, st);
  } else if (bm == 16) launch_gemm<16, 64, 1, 4>(g, batch, splits, st);
  else if (bm == 32 && bn == 32) launch_gemm<32, 32, 2, 2>(g, batch, splits, st);
  else if (bm == 32) launch_gemm<32, 128, 1, 4>(g, batch, splits, st);
  else if (bn == 16) launch_gemm<64, 16, 4, 1>(g, batch, splits, st);
  else if (bm == 128) launch_gemm<128, 32, 4, 1>(g, batch, splits, st);
  else if (bn == 32) launch_gemm<64, 32, 2, 2>(g, batch, splits, st);
  else launch_gemm<64, 64, 2, 2>(g, batch, splits, st);
  LS_HIP(hipGetLastError());
  return LS_OK;
}

GemmP gp(int M, int N, int K, const float* A, long long sam, long long sak, long long sab,
         const float* B, long long sbk, long long sbn, long long sbb, float* C, long long scm,
         long long scn, long long scb, float alpha = 1.f, float beta = 0.f,
         const float* bias = nullptr) {
  GemmP g{};
  g.M = M; g.N = N; g.K = K;
  g.A = A; g.sam = sam; g.sak = sak; g.sab = sab;
  g.B = B; g.sbk = sbk; g.sbn = sbn; g.sbb = sbb;
  g.C = C; g.scm = scm; g.scn = scn; g.scb = scb;
  g.alpha = alpha; g.beta = beta; g.bias_m = bias;
  return g;
}

// ----------------------------------------------------------- elementwise

// g *= GELU'(z)
__global__ void k_gelu_back(float* __restrict__ g, const float* __restrict__ z, size_t cnt) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += (size_t)gridDim.x * blockDim.x)
    g[i] *= gelu_d(z[i]);
}

// Output of Fourier layer l for one row j of one sample s, as one K = 64
// product on matrix cores:
//   z[s][o][j n + i] = sum_x' U[s][o][j][x'] Gx[x'][i] + sum_c W[o][c] v[s][c][j n + i] + b[o]
// (the inverse DFT along x of the mixed modes plus the pointwise map), then
// z is stored when requested and GELU(z) written as the next layer's input.
// A workgroup takes 32 outputs x kLBN pixels of the row; wave w owns
// pixels [32 w, 32 w + 32) as 2 x 2 tiles of 16 x 16 (16x16x32 bf16 MFMA).
constexpr int kLBN = 128;
__global__ __launch_bounds__(256) void k_layer_out(const float* __restrict__ U, const float* __restrict__ Gx,
                                                   const float* __restrict__ Wt, const float* __restrict__ bias,
                                                   const float* __restrict__ v, float* __restrict__ z,
                                                   float* __restrict__ vn, int n) {
  constexpr int K = 64, LDK = 72;
  __shared__ __attribute__((aligned(16))) __bf16 As[kW * LDK];
  __shared__ __attribute__((aligned(16))) __bf16 Bs[kLBN * LDK];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int i0 = blockIdx.x * kLBN, j = blockIdx.y, s = blockIdx.z;
  const long long P = (long long)n * n;
  for (int e = tid; e < kW * K; e += 256) {
    const int o = e / K, k = e % K;
    const float a = k < 32 ? U[(((long long)s * kW + o) * n + j) * 32 + k] : Wt[o * kW + (k - 32)];
    As[o * LDK + k] = (__bf16)a;
  }
  for (int e = tid; e < K * kLBN; e += 256) {
    const int k = e / kLBN, ii = e % kLBN, i = i0 + ii;  // pixels fastest: coalesced
    float b = 0.f;
    if (i < n)
      b = k < 32 ? Gx[(long long)k * n + i] : v[((long long)s * kW + (k - 32)) * P + (long long)j * n + i];
    Bs[ii * LDK + k] = (__bf16)b;
  }
  __syncthreads();
  const int r16 = lane & 15, kq = (lane >> 4) * 8;
  f32x4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int c = 0; c < 2; ++c) acc[a][c] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int ks = 0; ks < K; ks += 32) {
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      const bf16x8 av = *reinterpret_cast<const bf16x8*>(&As[(a * 16 + r16) * LDK + ks + kq]);
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        const bf16x8 bv = *reinterpret_cast<const bf16x8*>(&Bs[(wave * 32 + c * 16 + r16) * LDK + ks + kq]);
        acc[a][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc[a][c], 0, 0, 0);
      }
    }
  }
  // D layout: lane holds rows 4 (lane / 16) + t of column lane % 16
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int o = a * 16 + (lane >> 4) * 4 + t;
        const int i = i0 + wave * 32 + c * 16 + (lane & 15);
        if (i >= n) continue;
        const float val = acc[a][c][t] + bias[o];
        const long long idx = ((long long)s * kW + o) * P + (long long)j * n + i;
        if (z) z[idx] = val;
        if (vn) vn[idx] = gelu_f(val);
      }
}

// DFT tables for grid side n (angles in FP64, stored FP32):
//   Fx2[i][x]  = cos(2 pi x i / n),  Fx2[i][16 + x] = -sin(2 pi x i / n)
//   Gx[x][i]   = c_x cos(2 pi x i / n), Gx[16 + x][i] = -c_x sin(...)
//   Fa[k][j]   = cos(2 pi kz j / n), Fa[32 + k][j] = -sin(...)      (Re / Im of e^{-i..})
//   Fb[k][j]   = sin(2 pi kz j / n), Fb[32 + k][j] =  cos(...)
//   Ai[j][k]   = cos(2 pi kz j / n), Ai[j][32 + k] =  sin(...)      (Re / Im of e^{+i..})
//   FxH[x][i] = Fx2[i][x], GxH[i][x] = Gx[x][i] as bf16 (inference: the
//   operand layouts the matrix cores read with one 16-byte load per lane)
__global__ void k_tables(int n, float* Fx2, float* Gx, float* Fa, float* Fb, float* Ai, __bf16* FxH, __bf16* GxH) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  for (int x = 0; x < kM; ++x) {
    const long long ph = ((long long)x * j) % n;
    double s, c;
    sincospi(2.0 * (double)ph / n, &s, &c);
    const float cx = x == 0 ? 1.f : 2.f;
    Fx2[(size_t)j * 32 + x] = (float)c;
    Fx2[(size_t)j * 32 + kM + x] = (float)-s;
    Gx[(size_t)x * n + j] = cx * (float)c;
    Gx[(size_t)(kM + x) * n + j] = -cx * (float)s;
    FxH[(size_t)x * n + j] = (__bf16)(float)c;
    FxH[(size_t)(kM + x) * n + j] = (__bf16)(float)-s;
    GxH[(size_t)j * 32 + x] = (__bf16)(cx * (float)c);
    GxH[(size_t)j * 32 + kM + x] = (__bf16)(-cx * (float)s);
  }
  for (int k = 0; k < kKZ; ++k) {
    const int kz = k < kM ? k : k - kKZ;
    long long ph = ((long long)kz * j) % n;
    if (ph < 0) ph += n;
    double s, c;
    sincospi(2.0 * (double)ph / n, &s, &c);
    Fa[(size_t)k * n + j] = (float)c;
    Fa[(size_t)(kKZ + k) * n + j] = (float)-s;
    Fb[(size_t)k * n + j] = (float)s;
    Fb[(size_t)(kKZ + k) * n + j] = (float)c;
    Ai[(size_t)j * 64 + k] = (float)c;
    Ai[(size_t)j * 64 + kKZ + k] = (float)s;
  }
}

// Mode mixing, one workgroup per retained mode (k, x): Wh[s][o] =
// sum_c R[o][c] Vh[s][c], written as the 64 x 32 block operand
// [[Re, Im], [-Im, Re]] of the inverse kz transform.
// Vh: [S][32 c][64][16] (rows 0..31 real parts, 32..63 imaginary);
// Bst: [S][32 o][64][32].
__global__ __launch_bounds__(256) void k_modemix(const float* __restrict__ Vh, const float* __restrict__ Rre,
                                                 const float* __restrict__ Rim, float* __restrict__ Bst, int S) {
  const int mode = blockIdx.x, k = mode / kM, x = mode % kM;
  __shared__ float rr[kW * kW], ri[kW * kW];
  __shared__ float vr[8][kW], vi[8][kW];
  const size_t roff = (size_t)mode * kW * kW;
  for (int e = threadIdx.x; e < kW * kW; e += 256) {
    rr[e] = Rre[roff + e];
    ri[e] = Rim[roff + e];
  }
  const int o = threadIdx.x % kW, sl = threadIdx.x / kW;
  for (int s0 = 0; s0 < S; s0 += 8) {
    __syncthreads();
    {
      const int s = s0 + sl, c = o;
      if (s < S) {
        const size_t base = ((size_t)(s * kW + c) * 64) * kM;
        vr[sl][c] = Vh[base + (size_t)k * kM + x];
        vi[sl][c] = Vh[base + (size_t)(kKZ + k) * kM + x];
      }
    }
    __syncthreads();
    const int s = s0 + sl;
    if (s >= S) continue;
    float wr = 0.f, wi = 0.f;
    for (int c = 0; c < kW; ++c) {
      const float a = rr[o * kW + c], bq = ri[o * kW + c];
      wr = fmaf(a, vr[sl][c], fmaf(-bq, vi[sl][c], wr));
      wi = fmaf(a, vi[sl][c], fmaf(bq, vr[sl][c], wi));
    }
    float* B = Bst + (size_t)(s * kW + o) * 64 * 32;
    B[k * 32 + x] = wr;
    B[k * 32 + kM + x] = wi;
    B[(kKZ + k) * 32 + x] = -wi;
    B[(kKZ + k) * 32 + kM + x] = wr;
  }
}

// Adjoint of k_modemix for one mode: from dL/dBst to the complex gradient
// gW = dL/dRe Wh + i dL/dIm Wh, then dL/dVh = conj(R)^T gW (per sample) and
// dL/dR = sum_s gW conj(Vh)^T (written to the gradient vector).
__global__ __launch_bounds__(256) void k_modemix_back(const float* __restrict__ gB, const float* __restrict__ Vh,
                                                      const float* __restrict__ Rre, const float* __restrict__ Rim,
                                                      float* __restrict__ gVh, float* __restrict__ gRre,
                                                      float* __restrict__ gRim, int S) {
  const int mode = blockIdx.x, k = mode / kM, x = mode % kM;
  __shared__ float rr[kW * kW], ri[kW * kW];
  __shared__ float gwr[8][kW], gwi[8][kW], vr[8][kW], vi[8][kW];
  const size_t roff = (size_t)mode * kW * kW;
  for (int e = threadIdx.x; e < kW * kW; e += 256) {
    rr[e] = Rre[roff + e];
    ri[e] = Rim[roff + e];
  }
  // dL/dR accumulators: thread owns (o, c) pairs e = tid + 256 q, q < 4
  float ar[4] = {0, 0, 0, 0}, ai[4] = {0, 0, 0, 0};
  const int t = threadIdx.x % kW, sl = threadIdx.x / kW;
  for (int s0 = 0; s0 < S; s0 += 8) {
    __syncthreads();
    {
      const int s = s0 + sl;
      if (s < S) {
        const float* G = gB + (size_t)(s * kW + t) * 64 * 32;  // t plays o
        gwr[sl][t] = G[k * 32 + x] + G[(kKZ + k) * 32 + kM + x];
        gwi[sl][t] = G[k * 32 + kM + x] - G[(kKZ + k) * 32 + x];
        const size_t base = ((size_t)(s * kW + t) * 64) * kM;  // t plays c
        vr[sl][t] = Vh[base + (size_t)k * kM + x];
        vi[sl][t] = Vh[base + (size_t)(kKZ + k) * kM + x];
      } else {
        gwr[sl][t] = gwi[sl][t] = vr[sl][t] = vi[sl][t] = 0.f;
      }
    }
    __syncthreads();
    const int s = s0 + sl;
    if (s < S) {  // dL/dVh[s][c = t] = sum_o conj(R[o][c]) gW[o]
      float pr = 0.f, pi = 0.f;
      for (int o = 0; o < kW; ++o) {
        const float a = rr[o * kW + t], bq = ri[o * kW + t];
        pr = fmaf(a, gwr[sl][o], fmaf(bq, gwi[sl][o], pr));
        pi = fmaf(a, gwi[sl][o], fmaf(-bq, gwr[sl][o], pi));
      }
      const size_t base = ((size_t)(s * kW + t) * 64) * kM;
      gVh[base + (size_t)k * kM + x] = pr;
      gVh[base + (size_t)(kKZ + k) * kM + x] = pi;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = threadIdx.x + 256 * q, o = e / kW, c = e % kW;
      for (int ss = 0; ss < 8; ++ss) {  // gW conj(V)
        ar[q] = fmaf(gwr[ss][o], vr[ss][c], fmaf(gwi[ss][o], vi[ss][c], ar[q]));
        ai[q] = fmaf(gwi[ss][o], vr[ss][c], fmaf(-gwr[ss][o], vi[ss][c], ai[q]));
      }
    }
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int e = threadIdx.x + 256 * q;
    gRre[roff + e] = ar[q];
    gRim[roff + e] = ai[q];
  }
}

// gb[m] += sum over samples and points of g[s][m][p] (gb zeroed before).
__global__ void k_bias_grad(const float* __restrict__ g, int S, int Mc, size_t P, float* gb) {
  const int m = blockIdx.y;
  float acc = 0.f;
  const size_t cnt = (size_t)S * P;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < cnt; e += (size_t)gridDim.x * blockDim.x) {
    const size_t s = e / P, p = e % P;
    acc += g[(s * Mc + m) * P + p];
  }
  __shared__ float red[256];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicAdd(gb + m, red[0]);
}

__global__ void k_zero_f(float* a, size_t cnt) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += (size_t)gridDim.x * blockDim.x)
    a[i] = 0.f;
}

// Per-sample partial sums (FP64) of ||r||^2 over grid vectors [S][P] complex.
template <typename T>
__global__ void k_sq_partial(const T* __restrict__ r, size_t P, double* part) {
  const int s = blockIdx.y;
  double acc = 0.0;
  for (size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x; p < P; p += (size_t)gridDim.x * blockDim.x) {
    const T v = r[(size_t)s * P + p];
    acc += (double)v.x * v.x + (double)v.y * v.y;
  }
  __shared__ double red[256];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[(size_t)s * gridDim.x + blockIdx.x] = red[0];
}

// s[b] = sqrt(sum of partials) / n
__global__ void k_rms(const double* part, int nparts, int n, double* s, int S) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= S) return;
  double a = 0.0;
  for (int i = 0; i < nparts; ++i) a += part[(size_t)b * nparts + i];
  s[b] = sqrt(a) / n;
}

template <typename T>
__global__ void k_inputs(const double* __restrict__ m, size_t mstr, const cplx* __restrict__ uI,
                         const T* __restrict__ r, const double* __restrict__ s, float* __restrict__ x,
                         size_t P) {
  const int b = blockIdx.y;
  const double inv = s[b] > 0.0 ? 1.0 / s[b] : 0.0;
  for (size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x; p < P; p += (size_t)gridDim.x * blockDim.x) {
    const cplx u = uI[(size_t)b * P + p];
    const T rv = r[(size_t)b * P + p];
    float* xb = x + (size_t)b * kIn * P;
    xb[p] = (float)m[(size_t)b * mstr + p];
    xb[P + p] = (float)u.x;
    xb[2 * P + p] = (float)u.y;
    xb[3 * P + p] = (float)(rv.x * inv);
    xb[4 * P + p] = (float)(rv.y * inv);
  }
}

// Inference lift from the raw inputs: x = (m, Re uI, Im uI, Re r / s,
// Im r / s) as k_inputs forms it, then v0 = L x + b (32 channels, FP32
// products of the 5 inputs), stored as bf16, the precision in which the
// first Fourier layer's products read it.
template <typename T>
__global__ __launch_bounds__(256) void k_lift_in(const double* __restrict__ m, size_t mstr,
                                                 const cplx* __restrict__ uI, const T* __restrict__ r,
                                                 const double* __restrict__ s, const float* __restrict__ Lw,
                                                 const float* __restrict__ Lb, __bf16* __restrict__ v, size_t P) {
  __shared__ float w[kW * kIn + kW];
  for (int e = threadIdx.x; e < kW * kIn + kW; e += blockDim.x) w[e] = e < kW * kIn ? Lw[e] : Lb[e - kW * kIn];
  __syncthreads();
  const int b = blockIdx.y;
  const size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x;  // one pixel per thread
  if (p >= P) return;
  const double inv = s[b] > 0.0 ? 1.0 / s[b] : 0.0;
  __bf16* vb = v + (size_t)b * kW * P;
  const cplx u = uI[(size_t)b * P + p];
  const T rv = r[(size_t)b * P + p];
  const float x[kIn] = {(float)m[(size_t)b * mstr + p], (float)u.x, (float)u.y, (float)(rv.x * inv),
                        (float)(rv.y * inv)};
#pragma unroll 8
  for (int o = 0; o < kW; ++o) {
    float a = w[kW * kIn + o];
#pragma unroll
    for (int c = 0; c < kIn; ++c) a = fmaf(w[o * kIn + c], x[c], a);
    vb[(size_t)o * P + p] = (__bf16)a;
  }
}

// ------------------------------------------------------ inference kernels
// Activations are bf16 [S][32][P] (channel-major, as the training layout),
// read and written in runs of 8 pixels (16 bytes); the matrix-core operands
// that need 8 consecutive channels of one pixel are gathered from a tile
// staged in LDS.

// GELU with erf from Abramowitz & Stegun, Handbook of Mathematical
// Functions, formula 7.1.26 (absolute error in erf at most 1.5e-7), for
// inference, whose activations are then rounded to bf16 (relative spacing
// 2^-8); training uses the library erf (gelu_f).
__device__ __forceinline__ float gelu_as(float x) {
  const float y = fabsf(x) * 0.70710678118654752f;
  const float t = __builtin_amdgcn_rcpf(fmaf(0.3275911f, y, 1.f));
  const float q =
      t * fmaf(t, fmaf(t, fmaf(t, fmaf(t, 1.061405429f, -1.453152027f), 1.421413741f), -0.284496736f), 0.254829592f);
  const float e = 1.f - q * __expf(-y * y);  // erf(|x| / sqrt 2)
  return 0.5f * x * (1.f + copysignf(e, x));
}

typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));

// p[off .. off + 8) as bf16, zero from index `valid` on; one 16-byte load
// when the run is whole and `aligned` (off a multiple of 8).
__device__ __forceinline__ bf16x8 ld8(const __bf16* __restrict__ p, long long off, long long valid, bool aligned) {
  if (aligned && valid >= 8) return *reinterpret_cast<const bf16x8*>(p + off);
  bf16x8 r;
#pragma unroll
  for (int q = 0; q < 8; ++q) r[q] = q < valid ? p[off + q] : (__bf16)0.f;
  return r;
}

// 8 FP32 values (16-byte aligned) rounded to bf16
__device__ __forceinline__ bf16x8 f8_to_bf(const float* __restrict__ p) {
  const float4 a = *reinterpret_cast<const float4*>(p), b = *reinterpret_cast<const float4*>(p + 4);
  bf16x8 r;
  r[0] = (__bf16)a.x; r[1] = (__bf16)a.y; r[2] = (__bf16)a.z; r[3] = (__bf16)a.w;
  r[4] = (__bf16)b.x; r[5] = (__bf16)b.y; r[6] = (__bf16)b.z; r[7] = (__bf16)b.w;
  return r;
}

// LDS tile of 32 channels x 128 pixels, rows padded to kLDV bf16 (264
// bytes: 8-byte runs stay aligned, and the four lane groups of an operand
// gather (rows 8 apart) and of the output scatter (rows 4 apart) fall in
// distinct banks).
constexpr int kTP = 128, kLDV = 132;

// Stage v[c * P + base .. + kTP) for c < 32 (zero past `limit` pixels).
__device__ __forceinline__ void stage_tile(__bf16* Vs, const __bf16* __restrict__ v, long long P, long long base,
                                           long long limit, bool aligned, int tid) {
  for (int e = tid; e < kW * (kTP / 8); e += 256) {
    const int c = e / (kTP / 8), q8 = (e % (kTP / 8)) * 8;
    const bf16x8 x = ld8(v, (long long)c * P + base + q8, limit - q8, aligned);
    bf16x4* d = reinterpret_cast<bf16x4*>(&Vs[c * kLDV + q8]);
    d[0] = bf16x4{x[0], x[1], x[2], x[3]};
    d[1] = bf16x4{x[4], x[5], x[6], x[7]};
  }
}

// B operand of a K = 32 product over channels: channels kq .. kq + 7 of
// pixel column ii of the staged tile.
__device__ __forceinline__ bf16x8 gather8(const __bf16* Vs, int kq, int ii) {
  bf16x8 r;
#pragma unroll
  for (int q = 0; q < 8; ++q) r[q] = Vs[(kq + q) * kLDV + ii];
  return r;
}

// Write the staged output tile back: out[c * P + base + q8 ..] for the
// pixels below `limit`.
__device__ __forceinline__ void store_tile(__bf16* __restrict__ out, const __bf16* Vs, long long P, long long base,
                                           long long limit, bool aligned, int tid) {
  for (int e = tid; e < kW * (kTP / 8); e += 256) {
    const int c = e / (kTP / 8), q8 = (e % (kTP / 8)) * 8;
    const long long valid = limit - q8;
    if (valid <= 0) continue;
    const bf16x4* sp = reinterpret_cast<const bf16x4*>(&Vs[c * kLDV + q8]);
    const bf16x4 lo = sp[0], hi = sp[1];
    const bf16x8 x = {lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
    __bf16* d = out + (long long)c * P + base + q8;
    if (aligned && valid >= 8) {
      *reinterpret_cast<bf16x8*>(d) = x;
    } else {
#pragma unroll
      for (int q = 0; q < 8; ++q)
        if (q < valid) d[q] = x[q];
    }
  }
}

// x transform for inference: T[(s,c,j)][x'] = sum_i v[s][c][j n + i]
// Fx2[i][x'] (FP32 T, as the training forward).  One wave per (s, j)
// computes the 32 x 32 block D[x'][c] on matrix cores straight from global
// memory: A (x', 8 consecutive i) from the bf16 table FxH, B (8 consecutive
// i, channel c) from row j of channel c of v, one 16-byte load each (n a
// multiple of 8: rows start on 16-byte boundaries).
__global__ __launch_bounds__(256) void k_dftx_h(const __bf16* __restrict__ v, const __bf16* __restrict__ FxH,
                                                float* __restrict__ T, int n, int rows) {
  const int lane = threadIdx.x & 63;
  const int w = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (w >= rows) return;  // whole waves
  const int s = w / n, j = w % n;
  const long long P = (long long)n * n;
  const int r16 = lane & 15, g4 = lane >> 4, kq = g4 * 8;
  const __bf16* vb = v + (long long)s * kW * P + (long long)j * n;
  f32x4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int c = 0; c < 2; ++c) acc[a][c] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int i0 = 0; i0 < n; i0 += 32) {
    const int valid = n - (i0 + kq);
    bf16x8 a[2], b[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      a[q] = ld8(FxH, (long long)(16 * q + r16) * n + i0 + kq, valid, true);
      b[q] = ld8(vb, (long long)(16 * q + r16) * P + i0 + kq, valid, true);
    }
#pragma unroll
    for (int xb = 0; xb < 2; ++xb)
#pragma unroll
      for (int cb = 0; cb < 2; ++cb) acc[xb][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[xb], b[cb], acc[xb][cb], 0, 0, 0);
  }
  // lane holds D[x' = 16 xb + 4 g4 + t][c = 16 cb + r16]: 4 consecutive x'
#pragma unroll
  for (int xb = 0; xb < 2; ++xb)
#pragma unroll
    for (int cb = 0; cb < 2; ++cb) {
      const int c = 16 * cb + r16, x0 = 16 * xb + 4 * g4;
      *reinterpret_cast<float4*>(&T[(((long long)s * kW + c) * n + j) * 32 + x0]) =
          make_float4(acc[xb][cb][0], acc[xb][cb][1], acc[xb][cb][2], acc[xb][cb][3]);
    }
}

// Fourier layer output for inference: z = U Gx + W v + b for one row j of
// one sample and kTP pixels, as k_layer_out, then GELU(z) (or z for the
// last layer) in bf16.  The A operands (rows of U and W, 8 consecutive K)
// and the Gx operand (table GxH: 8 consecutive modes of one pixel) are
// 16-byte loads from global memory; v's operand (8 consecutive channels of
// one pixel) is gathered from the tile staged in LDS, which then holds the
// output tile for 16-byte stores.
__global__ __launch_bounds__(256) void k_layer_out_h(const float* __restrict__ U, const __bf16* __restrict__ GxH,
                                                     const float* __restrict__ Wt, const float* __restrict__ bias,
                                                     const __bf16* __restrict__ v, __bf16* __restrict__ out, int n,
                                                     int gelu) {
  __shared__ __attribute__((aligned(16))) __bf16 Vs[kW * kLDV];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int i0 = blockIdx.x * kTP, j = blockIdx.y, s = blockIdx.z;
  const long long P = (long long)n * n, base = (long long)s * kW * P + (long long)j * n + i0;
  const bool al = (n & 7) == 0;
  stage_tile(Vs, v + base, P, 0, n - i0, al, tid);
  const int r16 = lane & 15, g4 = lane >> 4, kq = g4 * 8;
  bf16x8 au[2], aw[2], bg[2];
#pragma unroll
  for (int a = 0; a < 2; ++a) {
    const int o = 16 * a + r16;
    au[a] = f8_to_bf(&U[(((long long)s * kW + o) * n + j) * 32 + kq]);
    aw[a] = f8_to_bf(&Wt[o * kW + kq]);
  }
#pragma unroll
  for (int cb = 0; cb < 2; ++cb) {
    const int i = i0 + 32 * wave + 16 * cb + r16;
    bg[cb] = i < n ? *reinterpret_cast<const bf16x8*>(&GxH[(long long)i * 32 + kq]) : bf16x8{};
  }
  __syncthreads();
  f32x4 acc[2][2];
#pragma unroll
  for (int cb = 0; cb < 2; ++cb) {
    const bf16x8 bv = gather8(Vs, kq, 32 * wave + 16 * cb + r16);
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      acc[a][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(au[a], bg[cb], f32x4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
      acc[a][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aw[a], bv, acc[a][cb], 0, 0, 0);
    }
  }
  __syncthreads();  // the tile is reused for the output
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int cb = 0; cb < 2; ++cb)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int o = 16 * a + 4 * g4 + t;
        const float val = acc[a][cb][t] + bias[o];
        Vs[o * kLDV + 32 * wave + 16 * cb + r16] = (__bf16)(gelu ? gelu_as(val) : val);
      }
  __syncthreads();
  store_tile(out + base, Vs, P, 0, n - i0, al, tid);
}

// Inference output head and residual map in one pass over the last
// Fourier layer's output v: hid = GELU(P1 v + b1) (128 channels, a K = 32
// product on matrix cores per 16 x 16 block), y = P2 hid + b2 (FP32 sums of
// the GELU values), z = r + s (y0 + i y1).  A workgroup takes kTP pixels of
// one sample (staged in LDS as in k_layer_out_h); wave w owns pixels
// [32 w, 32 w + 32) against all 128 hidden channels.  In a block a lane
// holds 4 hidden channels of one pixel (rows 4 (lane / 16) + t of column
// lane % 16), so each lane sums its share of the two 128-term projections
// and the four lane groups of a column finish the sums with lane shuffles.
template <typename T>
__global__ __launch_bounds__(256, 2) void k_head(const __bf16* __restrict__ v, const float* __restrict__ W1,
                                                 const float* __restrict__ b1, const float* __restrict__ W2,
                                                 const float* __restrict__ b2, const T* __restrict__ r,
                                                 const double* __restrict__ s, T* __restrict__ z, long long P) {
  __shared__ __attribute__((aligned(16))) __bf16 Vs[kW * kLDV];
  __shared__ float sb1[kH], sw2[kOut * kH];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const long long p0 = (long long)blockIdx.x * kTP;
  const int b = blockIdx.y;
  for (int e = tid; e < kH; e += 256) sb1[e] = b1[e];
  for (int e = tid; e < kOut * kH; e += 256) sw2[e] = W2[e];
  stage_tile(Vs, v + (long long)b * kW * P, P, p0, P - p0, (P & 7) == 0, tid);
  __syncthreads();
  const int r16 = lane & 15, g4 = lane >> 4, kq = g4 * 8;
  bf16x8 bv[2];
#pragma unroll
  for (int j = 0; j < 2; ++j) bv[j] = gather8(Vs, kq, 32 * wave + 16 * j + r16);
  float y0[2] = {0.f, 0.f}, y1[2] = {0.f, 0.f};
#pragma unroll 2
  for (int a = 0; a < kH / 16; ++a) {
    const bf16x8 av = f8_to_bf(&W1[(a * 16 + r16) * kW + kq]);
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const f32x4 acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv[j], f32x4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int h = a * 16 + g4 * 4 + t;
        const float g = gelu_as(acc[t] + sb1[h]);
        y0[j] = fmaf(sw2[h], g, y0[j]);
        y1[j] = fmaf(sw2[kH + h], g, y1[j]);
      }
    }
  }
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    y0[j] += __shfl_xor(y0[j], 16);
    y0[j] += __shfl_xor(y0[j], 32);
    y1[j] += __shfl_xor(y1[j], 16);
    y1[j] += __shfl_xor(y1[j], 32);
  }
  // lane group j < 2 writes the pixels of block column j
  if (g4 < 2) {
    const long long p = p0 + 32 * wave + 16 * g4 + r16;
    if (p < P) {
      const double sc = s[b];
      const T rv = r[b * P + p];
      T o;
      o.x = rv.x + sc * (double)((g4 ? y0[1] : y0[0]) + b2[0]);
      o.y = rv.y + sc * (double)((g4 ? y1[1] : y1[0]) + b2[1]);
      z[b * P + p] = o;
    }
  }
}

// loss partials per sample: sum (y - t)^2 and sum t^2 (FP64)
__global__ void k_loss_partial(const float* __restrict__ y, const float* __restrict__ t, size_t Q, double* part) {
  const int s = blockIdx.y;
  double a = 0.0, d = 0.0;
  for (size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x; p < Q; p += (size_t)gridDim.x * blockDim.x) {
    const double yv = y[(size_t)s * Q + p], tv = t[(size_t)s * Q + p];
    a += (yv - tv) * (yv - tv);
    d += tv * tv;
  }
  __shared__ double ra[256], rd[256];
  ra[threadIdx.x] = a;
  rd[threadIdx.x] = d;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      ra[threadIdx.x] += ra[threadIdx.x + w];
      rd[threadIdx.x] += rd[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[((size_t)s * gridDim.x + blockIdx.x) * 2] = ra[0];
    part[((size_t)s * gridDim.x + blockIdx.x) * 2 + 1] = rd[0];
  }
}

// dy = 2 (y - t) / (S ||t_s||^2)
__global__ void k_loss_grad(const float* __restrict__ y, const float* __restrict__ t, const double* __restrict__ sums,
                            float* __restrict__ dy, size_t Q, int S) {
  const int s = blockIdx.y;
  const double f = 2.0 / (S * sums[2 * s + 1]);
  for (size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x; p < Q; p += (size_t)gridDim.x * blockDim.x) {
    const size_t i = (size_t)s * Q + p;
    dy[i] = (float)(f * ((double)y[i] - (double)t[i]));
  }
}

__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m1,
                       float* __restrict__ m2, size_t cnt, float lr, float b1, float b2, float eps,
                       float c1, float c2) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += (size_t)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float a = b1 * m1[i] + (1.f - b1) * gi;
    const float v = b2 * m2[i] + (1.f - b2) * gi * gi;
    m1[i] = a;
    m2[i] = v;
    p[i] -= lr * (a / c1) / (sqrtf(v / c2) + eps);
  }
}

int grid_for(size_t cnt, int per = 256, int cap = 4096) {
  return (int)std::max<size_t>(1, std::min<size_t>(cap, (cnt + per - 1) / per));
}

}  // namespace

// ---------------------------------------------------------------- handle
struct FnoTables {
  float* Fx2 = nullptr;  // [n][32]
  float* Gx = nullptr;   // [32][n]
  float* Fa = nullptr;   // [64][n]
  float* Fb = nullptr;   // [64][n]
  float* Ai = nullptr;   // [n][64]
  __bf16* FxH = nullptr;  // [32][n] bf16
  __bf16* GxH = nullptr;  // [n][32] bf16
};

struct ls_fno {
  int max_batch = 0, max_n = 0, device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  float* params = nullptr;
  float* m1 = nullptr;
  float* m2 = nullptr;
  std::vector<size_t> off;  // offsets of the parameter blocks
  // activations, sized for max_batch x max_n^2
  float* v[kL] = {};        // layer inputs v_0..v_3 [S][32][P]
  float* z[kL] = {};        // pre-activations [S][32][P]; z[3] is v_4
  float* Vh[kL] = {};       // [S][32][64][16]
  float* hpre = nullptr;    // [S][128][P]
  float* hid = nullptr;     // [S][128][P]
  float* T = nullptr;       // [S][32][n][32] (also gT)
  float* U = nullptr;       // [S][32][n][32] (also gU)
  float* Bst = nullptr;     // [S][32][64][32] (also gBst)
  float* gVh = nullptr;     // [S][32][64][16]
  float* ga = nullptr;      // [S][32][P] gradient buffers
  float* gb = nullptr;
  float* x = nullptr;       // [S][5][P] (ls_fno_apply)
  float* y = nullptr;       // [S][2][P]
  double* s = nullptr;      // [S]
  double* part = nullptr;   // reduction scratch
  const float* xin = nullptr;  // inputs of the last keep = 1 forward
  int kept_n = 0, kept_S = 0;
  std::map<int, FnoTables> tables;
  std::vector<void*> allocs;
};

namespace {

enum ParamBlock { P_LIFT_W, P_LIFT_B, P_LAYER0 };
// block index of layer l, part q (0 spec re, 1 spec im, 2 w, 3 b)
inline int lb(int l, int q) { return P_LAYER0 + 4 * l + q; }
constexpr int P_PROJ1_W = P_LAYER0 + 4 * kL, P_PROJ1_B = P_PROJ1_W + 1, P_PROJ2_W = P_PROJ1_W + 2,
              P_PROJ2_B = P_PROJ1_W + 3;

std::vector<size_t> param_offsets() {
  std::vector<size_t> sz = {(size_t)kW * kIn, (size_t)kW};
  for (int l = 0; l < kL; ++l) {
    sz.push_back((size_t)kKZ * kM * kW * kW);
    sz.push_back((size_t)kKZ * kM * kW * kW);
    sz.push_back((size_t)kW * kW);
    sz.push_back((size_t)kW);
  }
  sz.push_back((size_t)kH * kW);
  sz.push_back((size_t)kH);
  sz.push_back((size_t)kOut * kH);
  sz.push_back((size_t)kOut);
  std::vector<size_t> off(sz.size() + 1, 0);
  for (size_t i = 0; i < sz.size(); ++i) off[i + 1] = off[i] + sz[i];
  return off;
}

ls_status fno_alloc(ls_fno* f, void** ptr, size_t bytes) {
  *ptr = nullptr;
  hipError_t e = hipMalloc(ptr, bytes ? bytes : 16);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    ls_set_error("hipMalloc of " + std::to_string(bytes) + " bytes failed: " + hipGetErrorString(e));
    *ptr = nullptr;
    return LS_ENOMEM;
  }
  f->allocs.push_back(*ptr);
  return LS_OK;
}

ls_status tables_for(ls_fno* f, int n, FnoTables** out) {
  auto it = f->tables.find(n);
  if (it == f->tables.end()) {
    FnoTables t;
    LS_TRY(fno_alloc(f, (void**)&t.Fx2, sizeof(float) * n * 32));
    LS_TRY(fno_alloc(f, (void**)&t.Gx, sizeof(float) * n * 32));
    LS_TRY(fno_alloc(f, (void**)&t.Fa, sizeof(float) * n * 128));  // Fa then Fb, adjacent
    t.Fb = t.Fa + (size_t)64 * n;
    LS_TRY(fno_alloc(f, (void**)&t.Ai, sizeof(float) * n * 64));
    LS_TRY(fno_alloc(f, (void**)&t.FxH, sizeof(__bf16) * n * 64));  // FxH then GxH
    t.GxH = t.FxH + (size_t)32 * n;
    k_tables<<<(n + 127) / 128, 128, 0, f->stream>>>(n, t.Fx2, t.Gx, t.Fa, t.Fb, t.Ai, t.FxH, t.GxH);
    LS_HIP(hipGetLastError());
    it = f->tables.emplace(n, t).first;
  }
  *out = &it->second;
  return LS_OK;
}

inline const float* par(const ls_fno* f, int blk) { return f->params + f->off[blk]; }

// Vh[s,c] = (Fa T_re + Fb T_im) / n^2: one product over K = 2n when n is a
// multiple of the K tile (Fa and Fb adjacent; the second K segment reads
// T's imaginary columns), else two products.
ls_status vh_gemm(ls_fno* f, const FnoTables* tb, int n, int S, float* Vh) {
  const float inv_n2 = 1.f / (float)((double)n * n);
  if (n % 32 == 0) {
    GemmP g = gp(64, kM, 2 * n, tb->Fa, n, 1, 0, f->T, 32, 1, (long long)n * 32, Vh, kM, 1, 64 * kM, inv_n2, 0.f);
    g.kseg = n;
    g.sag = (long long)64 * n;
    g.sbg = kM;
    return gemm(g, S * kW, f->stream);
  }
  LS_TRY(gemm(gp(64, kM, n, tb->Fa, n, 1, 0, f->T, 32, 1, (long long)n * 32, Vh, kM, 1, 64 * kM, inv_n2, 0.f),
              S * kW, f->stream));
  return gemm(gp(64, kM, n, tb->Fb, n, 1, 0, f->T + kM, 32, 1, (long long)n * 32, Vh, kM, 1, 64 * kM, inv_n2, 1.f),
              S * kW, f->stream);
}

// y = network(x); keep: store every activation for backward.
ls_status forward(ls_fno* f, int n, int S, const float* x, float* y, bool keep) {
  hipStream_t st = f->stream;
  FnoTables* tb;
  LS_TRY(tables_for(f, n, &tb));
  const long long P = (long long)n * n;
  // buffers: with keep every layer has its own v / z; without, two rotate
  float* vin = f->v[0];
  LS_TRY(gemm(gp(kW, (int)P, kIn, par(f, P_LIFT_W), kIn, 1, 0, x, P, 1, kIn * P, vin, P, 1, kW * P, 1.f, 0.f,
                 par(f, P_LIFT_B)), S, st));
  float* zl = nullptr;
  for (int l = 0; l < kL; ++l) {
    zl = keep ? f->z[l] : f->z[l % 2];
    float* Vh = keep ? f->Vh[l] : f->Vh[0];
    // T[(s,c,j)][x'] = sum_i v[(s,c,j)][i] Fx2[i][x']
    LS_TRY(gemm(gp(S * kW * n, 32, n, vin, n, 1, 0, tb->Fx2, 32, 1, 0, f->T, 32, 1, 0), 1, st));
    LS_TRY(vh_gemm(f, tb, n, S, Vh));
    k_modemix<<<kKZ * kM, 256, 0, st>>>(Vh, par(f, lb(l, 0)), par(f, lb(l, 1)), f->Bst, S);
    LS_HIP(hipGetLastError());
    // U[s,o] = Ai Bst[s,o]
    LS_TRY(gemm(gp(n, 32, 64, tb->Ai, 64, 1, 0, f->Bst, 32, 1, 64 * 32, f->U, 32, 1, (long long)n * 32), S * kW, st));
    // z = U Gx + W v + b and the next input GELU(z) in one pass; z itself is
    // kept for backward and as the last layer's output
    const bool last = l == kL - 1;
    float* vn = last ? nullptr : (keep ? f->v[l + 1] : f->v[(l + 1) % 2]);
    k_layer_out<<<dim3((n + kLBN - 1) / kLBN, n, S), 256, 0, st>>>(f->U, tb->Gx, par(f, lb(l, 2)), par(f, lb(l, 3)),
                                                                   vin, (keep || last) ? zl : nullptr, vn, n);
    LS_HIP(hipGetLastError());
    if (!last) vin = vn;
  }
  const float* v4 = zl;
  {  // hidden layer: hpre = P1 v4 + b1 (kept for backward), hid = GELU(hpre) in the same pass
    GemmP q = gp(kH, (int)P, kW, par(f, P_PROJ1_W), kW, 1, 0, v4, P, 1, kW * P, keep ? f->hpre : nullptr, P, 1,
                 kH * P, 1.f, 0.f, par(f, P_PROJ1_B));
    q.C2 = f->hid;
    LS_TRY(gemm(q, S, st));
  }
  LS_TRY(gemm(gp(kOut, (int)P, kH, par(f, P_PROJ2_W), kH, 1, 0, f->hid, P, 1, kH * P, y, P, 1, kOut * P, 1.f, 0.f,
                 par(f, P_PROJ2_B)), S, st));
  if (keep) {
    // backward needs x after the caller may have reused its buffer
    if (x != f->x)
      LS_HIP(hipMemcpyAsync(f->x, x, sizeof(float) * S * kIn * P, hipMemcpyDeviceToDevice, st));
    f->xin = f->x;
    f->kept_n = n;
    f->kept_S = S;
  } else {
    f->kept_n = f->kept_S = 0;
  }
  return LS_OK;
}

// dW[m][c] = sum_s sum_p g[s][m][p] a[s][c][p]  (K = S * P in P-long segments)
ls_status weight_grad(ls_fno* f, int Mr, int Nc, const float* g, const float* a, long long P, int S, float* out) {
  GemmP q = gp(Mr, Nc, (int)(P * S), g, P, 1, 0, a, 1, P, 0, out, Nc, 1, 0);
  q.kseg = (int)P;
  q.sag = (long long)Mr * P;
  q.sbg = (long long)Nc * P;
  return gemm(q, 1, f->stream);
}

ls_status bias_grad(ls_fno* f, const float* g, int S, int Mc, long long P, float* out) {
  k_zero_f<<<1, 256, 0, f->stream>>>(out, Mc);
  const int gx = grid_for((size_t)S * P, 256, 64);
  k_bias_grad<<<dim3(gx, Mc), 256, 0, f->stream>>>(g, S, Mc, (size_t)P, out);
  LS_HIP(hipGetLastError());
  return LS_OK;
}

ls_status backward(ls_fno* f, int n, int S, const float* dy, float* grad) {
  hipStream_t st = f->stream;
  FnoTables* tb;
  LS_TRY(tables_for(f, n, &tb));
  const long long P = (long long)n * n;
  const float inv_n2 = 1.f / (float)((double)n * n);
  auto G = [&](int blk) { return grad + f->off[blk]; };
  // projection 2
  LS_TRY(weight_grad(f, kOut, kH, dy, f->hid, P, S, G(P_PROJ2_W)));
  LS_TRY(bias_grad(f, dy, S, kOut, P, G(P_PROJ2_B)));
  // dL/dhid overwrites hid, whose last use (the projection-2 weight
  // gradient) is ordered before it on the stream
  LS_TRY(gemm(gp(kH, (int)P, kOut, par(f, P_PROJ2_W), 1, kH, 0, dy, P, 1, kOut * P, f->hid, P, 1, kH * P), S, st));
  const size_t hc = (size_t)S * kH * P;
  k_gelu_back<<<grid_for(hc), 256, 0, st>>>(f->hid, f->hpre, hc);
  LS_HIP(hipGetLastError());
  const float* v4 = f->z[kL - 1];
  LS_TRY(weight_grad(f, kH, kW, f->hid, v4, P, S, G(P_PROJ1_W)));
  LS_TRY(bias_grad(f, f->hid, S, kH, P, G(P_PROJ1_B)));
  float* gv = f->ga;
  float* gv2 = f->gb;
  LS_TRY(gemm(gp(kW, (int)P, kH, par(f, P_PROJ1_W), 1, kW, 0, f->hid, P, 1, kH * P, gv, P, 1, kW * P), S, st));
  const size_t ac = (size_t)S * kW * P;
  for (int l = kL - 1; l >= 0; --l) {
    if (l < kL - 1) {
      k_gelu_back<<<grid_for(ac), 256, 0, st>>>(gv, f->z[l], ac);
      LS_HIP(hipGetLastError());
    }
    const float* gz = gv;
    const float* vl = f->v[l];
    LS_TRY(weight_grad(f, kW, kW, gz, vl, P, S, G(lb(l, 2))));
    LS_TRY(bias_grad(f, gz, S, kW, P, G(lb(l, 3))));
    // pointwise path: gv2 = W^T gz
    LS_TRY(gemm(gp(kW, (int)P, kW, par(f, lb(l, 2)), 1, kW, 0, gz, P, 1, kW * P, gv2, P, 1, kW * P), S, st));
    // spectral path: gU = gz Gx^T
    LS_TRY(gemm(gp(S * kW * n, 32, n, gz, n, 1, 0, tb->Gx, 1, n, 0, f->U, 32, 1, 0), 1, st));
    // gBst = Ai^T gU
    LS_TRY(gemm(gp(64, 32, n, tb->Ai, 1, 64, 0, f->U, 32, 1, (long long)n * 32, f->Bst, 32, 1, 64 * 32), S * kW, st));
    k_modemix_back<<<kKZ * kM, 256, 0, st>>>(f->Bst, f->Vh[l], par(f, lb(l, 0)), par(f, lb(l, 1)), f->gVh,
                                             G(lb(l, 0)), G(lb(l, 1)), S);
    LS_HIP(hipGetLastError());
    // gT_re = Fa^T gVh / n^2, gT_im = Fb^T gVh / n^2
    LS_TRY(gemm(gp(n, kM, 64, tb->Fa, 1, n, 0, f->gVh, kM, 1, 64 * kM, f->T, 32, 1, (long long)n * 32, inv_n2),
                S * kW, st));
    LS_TRY(gemm(gp(n, kM, 64, tb->Fb, 1, n, 0, f->gVh, kM, 1, 64 * kM, f->T + kM, 32, 1, (long long)n * 32, inv_n2),
                S * kW, st));
    // gv2 += gT Fx2^T
    LS_TRY(gemm(gp(S * kW * n, n, 32, f->T, 32, 1, 0, tb->Fx2, 1, 32, 0, gv2, n, 1, 0, 1.f, 1.f), 1, st));
    std::swap(gv, gv2);
  }
  LS_TRY(weight_grad(f, kW, kIn, gv, f->xin, P, S, G(P_LIFT_W)));
  LS_TRY(bias_grad(f, gv, S, kW, P, G(P_LIFT_B)));
  return LS_OK;
}

template <typename T>
ls_status make_inputs_t(ls_fno* f, int n, int S, const double* m, size_t mstr, const double* uI, const T* r,
                        float* x, double* s) {
  const size_t P = (size_t)n * n;
  const int parts = 64;
  k_sq_partial<T><<<dim3(parts, S), 256, 0, f->stream>>>(r, P, f->part);
  k_rms<<<(S + 63) / 64, 64, 0, f->stream>>>(f->part, parts, n, s, S);
  k_inputs<T><<<dim3(grid_for(P, 256, 1024), S), 256, 0, f->stream>>>(m, mstr, reinterpret_cast<const cplx*>(uI),
                                                                        r, s, x, P);
  LS_HIP(hipGetLastError());
  return LS_OK;
}

ls_status check_sizes(const ls_fno* f, int n, int S) {
  if (!f || n < 32 || n > f->max_n || S < 1 || S > f->max_batch) {
    ls_set_error("ls_fno: n must be in [32, max_n] and batch in [1, max_batch]");
    return LS_EINVAL;
  }
  return LS_OK;
}

// Inference on S <= max_batch samples straight from the raw inputs to the
// residual map z = r + s (y0 + i y1): the scale s, the lift, the four
// Fourier layers with bf16 activations (the two buffers v[0], v[1] hold
// them at half their FP32 size) and the fused output head.  The same
// network as forward(); the lift and the last projection run in FP32
// instead of bf16 products.
template <typename T>
ls_status infer(ls_fno* f, int n, int S, const double* m, size_t mstr, const double* uI, const T* r, T* z) {
  hipStream_t st = f->stream;
  FnoTables* tb;
  LS_TRY(tables_for(f, n, &tb));
  const long long P = (long long)n * n;
  const int parts = 64;
  k_sq_partial<T><<<dim3(parts, S), 256, 0, st>>>(r, P, f->part);
  k_rms<<<(S + 63) / 64, 64, 0, st>>>(f->part, parts, n, f->s, S);
  __bf16* act[2] = {reinterpret_cast<__bf16*>(f->v[0]), reinterpret_cast<__bf16*>(f->v[1])};
  k_lift_in<T><<<dim3((unsigned)((P + 255) / 256), S), 256, 0, st>>>(m, mstr, reinterpret_cast<const cplx*>(uI), r,
                                                                 f->s, par(f, P_LIFT_W), par(f, P_LIFT_B), act[0],
                                                                 (size_t)P);
  LS_HIP(hipGetLastError());
  for (int l = 0; l < kL; ++l) {
    const __bf16* vin = act[l % 2];
    __bf16* vout = act[(l + 1) % 2];
    if (n % 8 == 0) {
      k_dftx_h<<<(S * n + 3) / 4, 256, 0, st>>>(vin, tb->FxH, f->T, n, S * n);
      LS_HIP(hipGetLastError());
    } else {  // rows off 16-byte boundaries: the generic product
      GemmP gt = gp(S * kW * n, 32, n, nullptr, n, 1, 0, tb->Fx2, 32, 1, 0, f->T, 32, 1, 0);
      gt.Ah = vin;
      LS_TRY(gemm(gt, 1, st));
    }
    LS_TRY(vh_gemm(f, tb, n, S, f->Vh[0]));
    k_modemix<<<kKZ * kM, 256, 0, st>>>(f->Vh[0], par(f, lb(l, 0)), par(f, lb(l, 1)), f->Bst, S);
    LS_HIP(hipGetLastError());
    LS_TRY(gemm(gp(n, 32, 64, tb->Ai, 64, 1, 0, f->Bst, 32, 1, 64 * 32, f->U, 32, 1, (long long)n * 32), S * kW, st));
    // the last layer's output is z itself (no GELU)
    k_layer_out_h<<<dim3((n + kTP - 1) / kTP, n, S), 256, 0, st>>>(f->U, tb->GxH, par(f, lb(l, 2)), par(f, lb(l, 3)),
                                                                  vin, vout, n, l < kL - 1);
    LS_HIP(hipGetLastError());
  }
  k_head<T><<<dim3((unsigned)((P + kTP - 1) / kTP), S), 256, 0, st>>>(
      act[kL % 2], par(f, P_PROJ1_W), par(f, P_PROJ1_B), par(f, P_PROJ2_W), par(f, P_PROJ2_B), r, f->s, z, P);
  LS_HIP(hipGetLastError());
  f->kept_n = f->kept_S = 0;
  return LS_OK;
}

}  // namespace

// Residual map for the solver (complex type T): z = r + s (y0 + i y1), for
// any number S of vectors (the network runs on max_batch at a time).
template <typename T>
ls_status fno_residual_map(ls_fno* f, int n, int S, const double* m, size_t mstr, const double* uI, const T* r,
                           T* z) {
  if (S < 1) return LS_EINVAL;
  LS_TRY(check_sizes(f, n, 1));
  const size_t P = (size_t)n * n;
  for (int b0 = 0; b0 < S; b0 += f->max_batch) {
    const int B = std::min(f->max_batch, S - b0);
    LS_TRY(infer<T>(f, n, B, m + b0 * mstr, mstr, uI + 2 * b0 * P, r + b0 * P, z + b0 * P));
  }
  return LS_OK;
}
template ls_status fno_residual_map<cplx>(ls_fno*, int, int, const double*, size_t, const double*, const cplx*, cplx*);
template ls_status fno_residual_map<fcplx>(ls_fno*, int, int, const double*, size_t, const double*, const fcplx*,
                                           fcplx*);

hipStream_t fno_swap_stream(ls_fno* f, hipStream_t s) {
  hipStream_t old = f->stream;
  f->stream = s;
  return old;
}
int fno_max_batch(const ls_fno* f) { return f->max_batch; }
int fno_max_n(const ls_fno* f) { return f->max_n; }

extern "C" {

size_t ls_fno_param_count(void) { return param_offsets().back(); }

ls_status ls_fno_destroy(ls_fno* f) {
  if (!f) return LS_EINVAL;
  (void)hipSetDevice(f->device);
  (void)hipStreamSynchronize(f->stream);
  for (void* p : f->allocs) (void)hipFree(p);
  if (f->own_stream) (void)hipStreamDestroy(f->stream);
  delete f;
  return LS_OK;
}

ls_status ls_fno_create(ls_fno** out, int max_batch, int max_n, hipStream_t stream) {
  if (!out || max_batch < 1 || max_n < 32 || max_n > 4096) {
    ls_set_error("ls_fno_create: need max_batch >= 1 and 32 <= max_n <= 4096");
    return LS_EINVAL;
  }
  *out = nullptr;
  ls_fno* f = new ls_fno();
  f->max_batch = max_batch;
  f->max_n = max_n;
  (void)hipGetDevice(&f->device);
  if (stream) {
    f->stream = stream;
  } else {
    if (hipStreamCreateWithFlags(&f->stream, hipStreamDefault) != hipSuccess) {
      delete f;
      ls_set_error("ls_fno_create: hipStreamCreate failed");
      return LS_EDEVICE;
    }
    f->own_stream = true;
  }
  f->off = param_offsets();
  const size_t np = f->off.back();
  const size_t S = max_batch, P = (size_t)max_n * max_n, n = max_n;
  auto fail = [&](ls_status s) {
    ls_fno_destroy(f);
    return s;
  };
  ls_status s;
#define FNO_ALLOC(ptr, count)                                                     \
  if ((s = fno_alloc(f, (void**)&(ptr), sizeof(*(ptr)) * (count))) != LS_OK) return fail(s)
  FNO_ALLOC(f->params, np);
  FNO_ALLOC(f->m1, np);
  FNO_ALLOC(f->m2, np);
  for (int l = 0; l < kL; ++l) {
    FNO_ALLOC(f->v[l], S * kW * P);
    FNO_ALLOC(f->z[l], S * kW * P);
    FNO_ALLOC(f->Vh[l], S * kW * 64 * kM);
  }
  FNO_ALLOC(f->hpre, S * kH * P);
  FNO_ALLOC(f->hid, S * kH * P);
  FNO_ALLOC(f->T, S * kW * n * 32);
  FNO_ALLOC(f->U, S * kW * n * 32);
  FNO_ALLOC(f->Bst, S * kW * 64 * 32);
  FNO_ALLOC(f->gVh, S * kW * 64 * kM);
  FNO_ALLOC(f->ga, S * kW * P);
  FNO_ALLOC(f->gb, S * kW * P);
  FNO_ALLOC(f->x, S * kIn * P);
  FNO_ALLOC(f->y, S * kOut * P);
  FNO_ALLOC(f->s, S);
  FNO_ALLOC(f->part, S * 64 * 2);
#undef FNO_ALLOC
  k_zero_f<<<grid_for(np), 256, 0, f->stream>>>(f->params, np);
  k_zero_f<<<grid_for(np), 256, 0, f->stream>>>(f->m1, np);
  k_zero_f<<<grid_for(np), 256, 0, f->stream>>>(f->m2, np);
  if (hipGetLastError() != hipSuccess || hipStreamSynchronize(f->stream) != hipSuccess) {
    ls_set_error("ls_fno_create: initialisation kernels failed");
    return fail(LS_EDEVICE);
  }
  *out = f;
  return LS_OK;
}

ls_status ls_fno_set_params(ls_fno* f, const float* params) {
  if (!f || !params) return LS_EINVAL;
  const size_t np = f->off.back();
  LS_HIP(hipMemcpyAsync(f->params, params, np * sizeof(float), hipMemcpyDeviceToDevice, f->stream));
  k_zero_f<<<grid_for(np), 256, 0, f->stream>>>(f->m1, np);
  k_zero_f<<<grid_for(np), 256, 0, f->stream>>>(f->m2, np);
  LS_HIP(hipGetLastError());
  LS_HIP(hipStreamSynchronize(f->stream));
  return LS_OK;
}

ls_status ls_fno_get_params(ls_fno* f, float* params) {
  if (!f || !params) return LS_EINVAL;
  LS_HIP(hipMemcpyAsync(params, f->params, f->off.back() * sizeof(float), hipMemcpyDeviceToDevice, f->stream));
  LS_HIP(hipStreamSynchronize(f->stream));
  return LS_OK;
}

ls_status ls_fno_make_inputs(ls_fno* f, int n, int batch, const double* m, size_t m_stride, const double* uI,
                             const double* r, float* x, double* s) {
  LS_TRY(check_sizes(f, n, batch));
  if (!m || !uI || !r || !x || !s) return LS_EINVAL;
  return make_inputs_t<cplx>(f, n, batch, m, m_stride, uI, reinterpret_cast<const cplx*>(r), x, s);
}

ls_status ls_fno_forward(ls_fno* f, int n, int batch, const float* x, float* y, int keep) {
  LS_TRY(check_sizes(f, n, batch));
  if (!x || !y) return LS_EINVAL;
  return forward(f, n, batch, x, y, keep != 0);
}

ls_status ls_fno_loss(ls_fno* f, int n, int batch, const float* y, const float* target, float* dy,
                      double* loss_host) {
  LS_TRY(check_sizes(f, n, batch));
  if (!y || !target || !dy || !loss_host) return LS_EINVAL;
  const size_t Q = (size_t)kOut * n * n;
  const int parts = 64;
  k_loss_partial<<<dim3(parts, batch), 256, 0, f->stream>>>(y, target, Q, f->part);
  LS_HIP(hipGetLastError());
  std::vector<double> h((size_t)batch * parts * 2);
  LS_HIP(hipMemcpyAsync(h.data(), f->part, h.size() * sizeof(double), hipMemcpyDeviceToHost, f->stream));
  LS_HIP(hipStreamSynchronize(f->stream));
  // per-sample totals on the host (the loss is needed there), then back to
  // the device for the gradient
  std::vector<double> tot(2 * batch, 0.0);
  double L = 0.0;
  for (int b = 0; b < batch; ++b) {
    for (int i = 0; i < parts; ++i) {
      tot[2 * b] += h[((size_t)b * parts + i) * 2];
      tot[2 * b + 1] += h[((size_t)b * parts + i) * 2 + 1];
    }
    if (!(tot[2 * b + 1] > 0.0)) {
      ls_set_error("ls_fno_loss: zero target");
      return LS_EINVAL;
    }
    L += tot[2 * b] / tot[2 * b + 1];
  }
  *loss_host = L / batch;
  LS_HIP(hipMemcpyAsync(f->part, tot.data(), tot.size() * sizeof(double), hipMemcpyHostToDevice, f->stream));
  k_loss_grad<<<dim3(grid_for(Q, 256, 1024), batch), 256, 0, f->stream>>>(y, target, f->part, dy, Q, batch);
  LS_HIP(hipGetLastError());
  LS_HIP(hipStreamSynchronize(f->stream));
  return LS_OK;
}

ls_status ls_fno_backward(ls_fno* f, int n, int batch, const float* dy, float* grad) {
  LS_TRY(check_sizes(f, n, batch));
  if (!dy || !grad) return LS_EINVAL;
  if (f->kept_n != n || f->kept_S != batch || !f->xin) {
    ls_set_error("ls_fno_backward: needs a keep = 1 forward on the same n and batch");
    return LS_EINVAL;
  }
  LS_TRY(backward(f, n, batch, dy, grad));
  f->kept_n = f->kept_S = 0;  // hid / hpre were overwritten
  return LS_OK;
}

ls_status ls_fno_adam(ls_fno* f, const float* grad, double lr, double beta1, double beta2, double eps, int t) {
  if (!f || !grad || t < 1 || !(lr > 0) || !(beta1 >= 0 && beta1 < 1) || !(beta2 >= 0 && beta2 < 1))
    return LS_EINVAL;
  const size_t np = f->off.back();
  const float c1 = (float)(1.0 - std::pow(beta1, t)), c2 = (float)(1.0 - std::pow(beta2, t));
  k_adam<<<grid_for(np), 256, 0, f->stream>>>(f->params, grad, f->m1, f->m2, np, (float)lr, (float)beta1,
                                              (float)beta2, (float)eps, c1, c2);
  LS_HIP(hipGetLastError());
  return LS_OK;
}

ls_status ls_fno_apply(ls_fno* f, int n, int batch, const double* m, size_t m_stride, const double* uI,
                       const double* r, double* z) {
  if (!m || !uI || !r || !z || r == z) return LS_EINVAL;
  LS_TRY(fno_residual_map<cplx>(f, n, batch, m, m_stride, uI, reinterpret_cast<const cplx*>(r),
                                reinterpret_cast<cplx*>(z)));
  LS_HIP(hipStreamSynchronize(f->stream));
  return LS_OK;
}

ls_status ls_bf16_gemm(int M, int N, int K, int batch, const float* A, long long sam, long long sak, long long sab,
                       const float* B, long long sbk, long long sbn, long long sbb, float* C, long long scm,
                       long long scn, long long scb, float alpha, float beta, hipStream_t stream) {
  if (M < 0 || N < 0 || K < 0 || batch < 0 || !A || !B || !C) return LS_EINVAL;
  return gemm(gp(M, N, K, A, sam, sak, sab, B, sbk, sbn, sbb, C, scm, scn, scb, alpha, beta), batch, stream);
}

}  // extern "C"
