/* Learned preconditioner / warm start for the Lippmann-Schwinger solver:
 * a Fourier neural operator (FNO) evaluated and trained by the library's own
 * HIP kernels (bf16 MFMA products with FP32 accumulation).
 *
 * The paper's outer solver is flexible GMRES (Section 6), which accepts a
 * preconditioner that changes between iterations; the network below is used
 * as such a preconditioner and as an initial guess.  The paper itself has no
 * learned part: the architecture is the Fourier neural operator of Li et al.
 * (ICLR 2021) at a fixed size:
 *
 *   inputs per grid point  x = (m, Re u_I, Im u_I, Re r / s, Im r / s),
 *                          s = ||r||_2 / n (root-mean-square of r);
 *   lift                   v_0 = P x + p                      (5 -> 32);
 *   Fourier layer l=0..3   z_l = K_l v_l + W_l v_l + b_l,
 *                          v_{l+1} = GELU(z_l) (l < 3), v_4 = z_3;
 *   K_l                    truncated spectral convolution: forward DFT
 *                          with 1/n^2 on the modes kx = 0..15 and
 *                          kz = -16..15, one complex 32 x 32 matrix per
 *                          mode, inverse as the real part of the
 *                          half-spectrum sum (weight 1 at kx = 0, else 2);
 *   projection             y = Q2 GELU(Q1 v_4 + q1) + q2      (32 -> 128 -> 2);
 *   output                 z = r + s (y_0 + i y_1).
 *
 * GELU is the erf form x * Phi(x).
 *
 * Flat FP32 parameter vector (LS_FNO_PARAMS floats), in order:
 *   lift weight [32][5], lift bias [32];
 *   per layer l: spectral real part [32 kz][16 kx][32 out][32 in],
 *                spectral imaginary part (same shape),
 *                pointwise weight [32 out][32 in], bias [32];
 *   projection 1 weight [128][32], bias [128];
 *   projection 2 weight [2][128], bias [2].
 * The kz index k stands for kz = k (k < 16) and kz = k - 32 (k >= 16).
 *
 * Layouts: activations [batch][channel][n][n] FP32 with x fastest; grid
 * vectors (m, u_I, r, z) as in ls.h ([n][n], complex interleaved FP64).
 * Every pointer argument is a device pointer unless stated otherwise; all
 * work is enqueued on the stream given at creation.  A handle is not
 * re-entrant.
 */
#ifndef LS_FNO_H
#define LS_FNO_H

#include "ls.h"

#ifdef __cplusplus
extern "C" {
#endif

#define LS_FNO_WIDTH 32
#define LS_FNO_MODES 16
#define LS_FNO_LAYERS 4
#define LS_FNO_HIDDEN 128
#define LS_FNO_PARAMS 4203202

/* Modes of ls_solve_fno (bit set). */
#define LS_FNO_WARM 1  /* initial guess u0 = FNO(m, u_I, f) */
#define LS_FNO_PREC 2  /* FNO as the flexible-GMRES preconditioner */
#define LS_FNO_PROBE 4 /* with LS_FNO_WARM: the first right-hand side of the call is tried alone; if its
                        * warm start is dropped, the network is not evaluated for the others (same
                        * medium and grid) and no FNO-preconditioned pass runs */

/* Bits of ls_solve_info.fno_flags. */
#define LS_FNO_WARM_USED 1      /* the warm start was kept */
#define LS_FNO_WARM_REJECTED 2  /* the warm start was worse than u0 = 0 (or not finite): dropped */
#define LS_FNO_PREC_USED 4      /* the FNO-preconditioned pass was kept */
#define LS_FNO_PREC_FALLBACK 8  /* it stagnated: its correction was dropped, BD finished the solve */
#define LS_FNO_WARM_SKIPPED 16  /* LS_FNO_PROBE: the probe's warm start was dropped, the network was not
                                 * evaluated for this right-hand side (u0 = 0) */

typedef struct ls_fno ls_fno;

/* Number of FP32 parameters (LS_FNO_PARAMS). */
size_t ls_fno_param_count(void);

/* Allocates a network for up to max_batch samples on grids up to max_n x
 * max_n (n >= 32), its parameters (zero), gradient-free Adam moments and the
 * activation workspace (about 40 * max_batch * max_n^2 floats); stream NULL
 * makes the handle create its own blocking stream.  LS_ENOMEM if the device
 * memory is not there, LS_EINVAL for bad sizes. */
ls_status ls_fno_create(ls_fno** out, int max_batch, int max_n, hipStream_t stream);
ls_status ls_fno_destroy(ls_fno* f);

/* Copy LS_FNO_PARAMS floats in / out (device pointers).  set also clears the
 * Adam moments. */
ls_status ls_fno_set_params(ls_fno* f, const float* params);
ls_status ls_fno_get_params(ls_fno* f, float* params);

/* x [batch][5][n][n] and s [batch] (FP64) from a medium m (sample b reads
 * m + b * m_stride, m_stride = 0 shares one medium), incident fields
 * uI [batch][n][n] and residuals r [batch][n][n] (complex FP64).  A zero
 * residual gives s = 0 and zero residual channels. */
ls_status ls_fno_make_inputs(ls_fno* f, int n, int batch, const double* m, size_t m_stride,
                             const double* uI, const double* r, float* x, double* s);

/* y [batch][2][n][n] = network(x).  keep = 1 stores the activations that
 * ls_fno_backward needs (training); keep = 0 reuses the buffers. */
ls_status ls_fno_forward(ls_fno* f, int n, int batch, const float* x, float* y, int keep);

/* Relative loss L = mean_b ||y_b - t_b||^2 / ||t_b||^2 (returned on the
 * host, FP64 sums) and dL/dy into dy [batch][2][n][n].  LS_EINVAL if a
 * target is zero. */
ls_status ls_fno_loss(ls_fno* f, int n, int batch, const float* y, const float* target,
                      float* dy, double* loss_host);

/* grad [LS_FNO_PARAMS] = dL/dtheta for the dL/dy given, through the
 * activations of the last ls_fno_forward(keep = 1) on the same n and batch
 * (LS_EINVAL otherwise).  Overwrites grad. */
ls_status ls_fno_backward(ls_fno* f, int n, int batch, const float* dy, float* grad);

/* One Adam step (Kingma & Ba) on the parameters with gradient grad;
 * t >= 1 counts the steps since ls_fno_set_params. */
ls_status ls_fno_adam(ls_fno* f, const float* grad, double lr, double beta1, double beta2,
                      double eps, int t);

/* z = r + s (y_0 + i y_1) with y = network(make_inputs(m, uI, r)): the
 * network as a map from residuals to approximations of H^{-1} r.  z and r
 * complex FP64 [batch][n][n]; z may not alias r.  Any batch >= 1: the
 * network runs on max_batch vectors at a time. */
ls_status ls_fno_apply(ls_fno* f, int n, int batch, const double* m, size_t m_stride,
                       const double* uI, const double* r, double* z);

/* C = alpha op(A) op(B) + beta C on bf16-rounded operands with FP32
 * accumulation (MFMA), batched: element (m, k) of A is
 * A[b*sab + m*sam + k*sak], (k, n) of B is B[b*sbb + k*sbk + n*sbn], (m, n)
 * of C is C[b*scb + m*scm + n*scn].  FP32 storage.  The utility behind every
 * product of the network; exported for tests. */
ls_status ls_bf16_gemm(int M, int N, int K, int batch, const float* A, long long sam,
                       long long sak, long long sab, const float* B, long long sbk,
                       long long sbn, long long sbb, float* C, long long scm, long long scn,
                       long long scb, float alpha, float beta, hipStream_t stream);

/* ls_solve with the network (modes LS_FNO_WARM | LS_FNO_PREC | LS_FNO_PROBE) for the plan's
 * medium and the incident fields uI [batch][n][n] that produced f.  The
 * plain two-level preconditioner stays the fallback: a warm start whose
 * residual is not below ||f|| is dropped; an FNO-preconditioned pass that
 * does not halve the residual within max_outer / 4 iterations is dropped
 * and the solve continues with BD.  info[b].fno_flags reports what
 * happened.  n must be in the network's range; the network is evaluated
 * max_batch (its own) vectors at a time. */
ls_status ls_solve_fno(ls_plan* p, ls_fno* f, const double* uI, const double* fvec, double* u,
                       int batch, double tol, int mode, ls_solve_info* info);

/* Several media at once, as ls_solve_multi: one host thread per plan runs
 * ls_solve_fno(plans[i], fnos[i], ...) on that plan's stream.  Plans,
 * networks and streams must be distinct (a network handle is not
 * re-entrant); uI[i], f[i], u[i] device arrays of batch[i] grid vectors,
 * info[i] host arrays or info == NULL.  Returns the first failure. */
ls_status ls_solve_fno_multi(ls_plan* const* plans, ls_fno* const* fnos, int count,
                             const double* const* uI, const double* const* f, double* const* u,
                             const int* batch, double tol, int mode, ls_solve_info* const* info);

#ifdef __cplusplus
}
#endif

#endif /* LS_FNO_H */
