// Quadrature weights of the Green's function, FP64 on the device.
//
// Section 1, eq. (Greens_function): G(x) = -(i/4) H_0^(1)(omega |x|).
// Section 2: w_q = h^2 G(h |q|) for q != 0 (trapezoidal rule) and a
// modified diagonal weight w_0 (computed on the host from its closed form
// and passed in).
//
// J0 and Y0 are computed here from published expansions (no vendor Bessel
// routine):
//  * x < 25: Miller's backward recurrence J_{k-1} = (2k/x) J_k - J_{k+1}
//    (DLMF 10.74(iv)) normalised by 1 = J0 + 2 sum_{k>=1} J_{2k}
//    (DLMF 10.12), and Neumann's series
//    Y0 = (2/pi)(ln(x/2) + gamma) J0 - (4/pi) sum_{k>=1} (-1)^k J_{2k}/k
//    (DLMF 10.23).
//  * x >= 25: Hankel's asymptotic expansion (DLMF 10.17.3),
//    J0 = sqrt(2/(pi x)) (P cos chi - Q sin chi),
//    Y0 = sqrt(2/(pi x)) (P sin chi + Q cos chi), chi = x - pi/4, with
//    P = sum (-1)^k c_{2k} x^{-2k}, Q = -sum (-1)^k c_{2k+1} x^{-2k-1},
//    c_k = prod_{j<=k} (2j-1)^2 / (k! 8^k); at x >= 25 the terms fall below
//    1e-17 long before the series starts to diverge.
#include "ls_internal.h"

#include <cmath>

namespace {

constexpr double kEulerGamma = 0.57721566490153286060651209008240243;
constexpr double kTwoOverPi = 0.63661977236758134307553505349005745;
constexpr double kPi = 3.14159265358979323846264338327950288;

__device__ void bessel_j0_y0(double x, double& j0, double& y0) {
  if (x < 25.0) {
    const int N = 2 * static_cast<int>(x * 0.5) + 44;
    double jp1 = 0.0, j = 1e-250;
    double se = 0.0, sy = 0.0;
    for (int k = N; k >= 1; --k) {
      const double jm1 = (2.0 * k / x) * j - jp1;
      jp1 = j;
      j = jm1;  // j = J_{k-1}, jp1 = J_k (unnormalised)
      if ((k & 1) == 0) {
        se += jp1;
        const int mm = k >> 1;
        sy += ((mm & 1) ? -jp1 : jp1) / mm;
      }
      if (fabs(j) > 1e200) {
        j *= 1e-200;
        jp1 *= 1e-200;
        se *= 1e-200;
        sy *= 1e-200;
      }
    }
    const double norm = j + 2.0 * se;
    j0 = j / norm;
    y0 = kTwoOverPi * ((log(0.5 * x) + kEulerGamma) * j0 - 2.0 * sy / norm);
    return;
  }
  double t = 1.0, P = 1.0, Q = 0.0;
  for (int k = 1; k < 60; ++k) {
    t *= (double)((2 * k - 1) * (2 * k - 1)) / (8.0 * k * x);
    if ((k & 1) == 0) {
      P += ((k >> 1) & 1) ? -t : t;
    } else {
      Q -= (((k - 1) >> 1) & 1) ? -t : t;
    }
    if (t < 1e-17) break;
  }
  double s, c;
  sincos(x, &s, &c);
  const double r2 = 0.70710678118654752440084436210484904;
  const double cm = (c + s) * r2;  // cos(x - pi/4)
  const double sm = (s - c) * r2;  // sin(x - pi/4)
  const double f = sqrt(kTwoOverPi / x);
  j0 = f * (P * cm - Q * sm);
  y0 = f * (P * sm + Q * cm);
}

// w(qx, qz) for q != 0: h^2 * (-(i/4)) * (J0 + i Y0) = (h^2/4) (Y0, -J0).
__device__ __forceinline__ cplx weight(int qx, int qz, double oh, double hh4, cplx w0) {
  if (qx == 0 && qz == 0) return w0;
  const double rho = sqrt((double)qx * (double)qx + (double)qz * (double)qz);
  double j0, y0;
  bessel_j0_y0(oh * rho, j0, y0);
  return cmk(hh4 * y0, -hh4 * j0);
}

// c[y][x], P x P: the circulant embedding of w (zero where |q| > n-1).
__global__ void k_circulant(cplx* __restrict__ c, int n, int P, double oh, double hh4, cplx w0) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y;
  if (x >= P) return;
  int qx, qz;
  bool ok = true;
  if (x <= n - 1) qx = x; else if (x >= P - (n - 1)) qx = x - P; else { qx = 0; ok = false; }
  if (y <= n - 1) qz = y; else if (y >= P - (n - 1)) qz = y - P; else { qz = 0; ok = false; }
  c[(size_t)y * P + x] = ok ? weight(qx, qz, oh, hh4, w0) : cmk(0.0, 0.0);
}

__global__ void k_samples(cplx* __restrict__ w, int n, double oh, double hh4, cplx w0) {
  const int W = 2 * n - 1;
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y;
  if (x >= W) return;
  w[(size_t)y * W + x] = weight(x - (n - 1), y - (n - 1), oh, hh4, w0);
}

// Diagonal weight (Section 2, modified trapezoidal rule): the regular part
// of G at 0, -(i/4) + (ln(omega/2) + gamma)/(2 pi), plus the lattice
// correction (ln h + c_L)/(2 pi) of the (1/(2 pi)) ln r singularity, with
// c_L = ln(2 sqrt(pi) / Gamma(1/4)^2); all times h^2.
cplx diagonal_weight(double h, double omega) {
  const double cL = std::log(2.0 * std::sqrt(kPi) / (std::tgamma(0.25) * std::tgamma(0.25)));
  const double re = (std::log(omega * h / 2.0) + kEulerGamma + cL) / (2.0 * kPi);
  return cmk(h * h * re, h * h * -0.25);
}

}  // namespace

ls_status launch_circulant(ls_plan* p, cplx* c) {
  const double oh = p->omega * p->h;
  const double hh4 = 0.25 * (p->h * p->h);
  dim3 grid((p->P + 255) / 256, p->P);
  k_circulant<<<grid, 256, 0, p->stream>>>(c, p->n, p->P, oh, hh4, diagonal_weight(p->h, p->omega));
  LS_HIP(hipGetLastError());
  return LS_OK;
}

ls_status launch_kernel_samples(ls_plan* p, cplx* w) {
  const int W = 2 * p->n - 1;
  const double oh = p->omega * p->h;
  const double hh4 = 0.25 * (p->h * p->h);
  dim3 grid((W + 255) / 256, W);
  k_samples<<<grid, 256, 0, p->stream>>>(w, p->n, oh, hh4, diagonal_weight(p->h, p->omega));
  LS_HIP(hipGetLastError());
  return LS_OK;
}
