"""Fourier-neural-operator (FNO) preconditioner / warm start: FP64 reference.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The paper stops at flexible GMRES with the two-level preconditioner
(Section 6 names FGMRES, which admits any preconditioner that changes from
one iteration to the next).  It says nothing about learned components; this
module is the plain definition of the small network that the GPU path trains
and evaluates, written with explicit DFT matrices and NumPy contractions so
that each step can be read off.  The network is the Fourier neural operator
of Li et al. (2021): a pointwise lift, Fourier layers (truncated spectral
convolution plus a pointwise linear map, then GELU) and a pointwise
projection.  Readings (the architecture beyond "4 Fourier layers, width 32,
16 modes per axis, inputs (m, Re/Im u_I, Re/Im r)" is not fixed anywhere):

* Inputs per grid point: x = (m, Re u_I, Im u_I, Re r / s, Im r / s) with
  s = ||r||_2 / n the root-mean-square of the residual, so the network sees
  residuals of unit size whatever their scale.
* Lift 5 -> 32 (affine), L = 4 Fourier layers of width 32, GELU (erf form)
  after every layer but the last, projection 32 -> 128 (affine, GELU)
  -> 2 (affine).
* Truncated spectrum: kx = 0..M-1 (the real-input half), kz = 0..M-1 and
  -M..-1 (both corners), M = 16.  Forward transform with 1/n^2, inverse
  without, so that the same weights act on the same physical frequencies at
  every n.  The inverse is the real part of the half-spectrum sum with
  weight 1 for kx = 0 and 2 for kx > 0 (what an inverse real FFT does with
  the retained modes).
* Mode mixing: one complex C x C matrix per retained mode (kz, kx).
* Output: the network's two channels y are a correction in units of s:
  z = r + s (y_0 + i y_1).  Zero weights in the last projection give z = r.

All arrays are float64 / complex128; activations are [S][C][n][n] with the
x index fastest (the grid layout of ls_inputs).
"""
from __future__ import annotations

import numpy as np
from scipy.special import erf

WIDTH, MODES, LAYERS, HIDDEN, IN_CH, OUT_CH = 32, 16, 4, 128, 5, 2


def param_shapes(width=WIDTH, modes=MODES, layers=LAYERS, hidden=HIDDEN):
    """Names and shapes of the parameters, in the order of the flat vector.

    Spectral weights are stored as R[kz index][kx][out][in], real and
    imaginary parts as separate blocks (kz index k < M is kz = k, k >= M is
    kz = k - 2M)."""
    shapes = [("lift_w", (width, IN_CH)), ("lift_b", (width,))]
    for l in range(layers):
        shapes += [(f"spec_re{l}", (2 * modes, modes, width, width)),
                   (f"spec_im{l}", (2 * modes, modes, width, width)),
                   (f"w{l}", (width, width)), (f"b{l}", (width,))]
    shapes += [("proj1_w", (hidden, width)), ("proj1_b", (hidden,)),
               ("proj2_w", (OUT_CH, hidden)), ("proj2_b", (OUT_CH,))]
    return shapes


def flatten(params, **arch):
    return np.concatenate([np.asarray(params[k], dtype=np.float64).reshape(-1)
                           for k, _ in param_shapes(**arch)])


def unflatten(vec, **arch):
    out, o = {}, 0
    for k, shp in param_shapes(**arch):
        size = int(np.prod(shp))
        out[k] = np.asarray(vec[o:o + size], dtype=np.float64).reshape(shp)
        o += size
    assert o == len(vec), "flat parameter vector has the wrong length"
    return out


def gelu(x):
    """GELU(x) = x Phi(x) with the standard normal CDF Phi (erf form)."""
    return 0.5 * x * (1.0 + erf(x / np.sqrt(2.0)))


def gelu_grad(x):
    return 0.5 * (1.0 + erf(x / np.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / np.sqrt(2.0 * np.pi)


def kz_values(modes=MODES):
    return np.concatenate([np.arange(modes), np.arange(-modes, 0)])


def dft_tables(n, modes=MODES):
    """Fx[i, kx] = exp(-2 pi i kx i / n); Fz[k, j] = exp(-2 pi i kz(k) j / n)."""
    idx = np.arange(n)
    Fx = np.exp(-2j * np.pi * np.outer(idx, np.arange(modes)) / n)
    Fz = np.exp(-2j * np.pi * np.outer(kz_values(modes), idx) / n)
    cx = np.where(np.arange(modes) == 0, 1.0, 2.0)
    return Fx, Fz, cx


def spectral_forward(v, R, modes=MODES):
    """Truncated spectral convolution of real v [S][C][n][n] with complex
    mode matrices R [2M][M][O][C]."""
    n = v.shape[-1]
    Fx, Fz, cx = dft_tables(n, modes)
    Vh = np.einsum("kj,scji,ix->sckx", Fz, v, Fx) / n**2           # [S][C][2M][M]
    Wh = np.einsum("kxoc,sckx->sokx", R, Vh)                         # [S][O][2M][M]
    U = np.einsum("kj,sokx->sojx", np.conj(Fz), Wh)                  # [S][O][n][M]
    w = np.einsum("sojx,x,ix->soji", U, cx, np.conj(Fx)).real
    return w, Vh


def spectral_backward(gw, Vh, R, modes=MODES):
    """Adjoint of spectral_forward: from dL/dw (real) to dL/dv (real) and the
    complex gradient dL/dRe R + i dL/dIm R."""
    n = gw.shape[-1]
    Fx, Fz, cx = dft_tables(n, modes)
    gU = np.einsum("soji,x,ix->sojx", gw, cx, Fx)                    # complex gradient of U
    gWh = np.einsum("kj,sojx->sokx", Fz, gU)
    gR = np.einsum("sokx,sckx->kxoc", gWh, np.conj(Vh))
    gVh = np.einsum("kxoc,sokx->sckx", np.conj(R), gWh)
    gv = (np.einsum("sckx,kj,ix->scji", np.conj(gVh), Fz, Fx) / n**2).real
    return gv, gR


def pointwise(Wt, b, v):
    """y[s, o, p] = sum_c W[o, c] v[s, c, p] + b[o]."""
    return np.einsum("oc,scji->soji", Wt, v) + b[None, :, None, None]


def forward(params, x, modes=MODES, layers=LAYERS):
    """Network output y [S][2][n][n] for inputs x [S][5][n][n]; also returns
    the cache of intermediate values that backward needs."""
    cache = {"x": x}
    v = pointwise(params["lift_w"], params["lift_b"], x)
    for l in range(layers):
        R = params[f"spec_re{l}"] + 1j * params[f"spec_im{l}"]
        ws, Vh = spectral_forward(v, R, modes)
        z = ws + pointwise(params[f"w{l}"], params[f"b{l}"], v)
        cache[f"v{l}"], cache[f"Vh{l}"], cache[f"z{l}"] = v, Vh, z
        v = gelu(z) if l < layers - 1 else z
    cache["v_last"] = v
    hpre = pointwise(params["proj1_w"], params["proj1_b"], v)
    hid = gelu(hpre)
    cache["hpre"], cache["hid"] = hpre, hid
    y = pointwise(params["proj2_w"], params["proj2_b"], hid)
    return y, cache


def _pointwise_grads(gy, v, Wt):
    gW = np.einsum("soji,scji->oc", gy, v)
    gb = gy.sum(axis=(0, 2, 3))
    gv = np.einsum("oc,soji->scji", Wt, gy)
    return gW, gb, gv


def backward(params, cache, gy, modes=MODES, layers=LAYERS):
    """Gradients of a scalar loss with respect to every parameter, given
    dL/dy; by the chain rule through forward (analytic adjoint)."""
    g = {}
    g["proj2_w"], g["proj2_b"], ghid = _pointwise_grads(gy, cache["hid"], params["proj2_w"])
    ghpre = ghid * gelu_grad(cache["hpre"])
    g["proj1_w"], g["proj1_b"], gv = _pointwise_grads(ghpre, cache["v_last"], params["proj1_w"])
    for l in reversed(range(layers)):
        gz = gv * gelu_grad(cache[f"z{l}"]) if l < layers - 1 else gv
        R = params[f"spec_re{l}"] + 1j * params[f"spec_im{l}"]
        gv_s, gR = spectral_backward(gz, cache[f"Vh{l}"], R, modes)
        g[f"spec_re{l}"], g[f"spec_im{l}"] = gR.real, gR.imag
        g[f"w{l}"], g[f"b{l}"], gv_w = _pointwise_grads(gz, cache[f"v{l}"], params[f"w{l}"])
        gv = gv_s + gv_w
    g["lift_w"], g["lift_b"], _ = _pointwise_grads(gv, cache["x"], params["lift_w"])
    return g


def loss_rel(y, ystar):
    """Mean over the batch of ||y - y*||^2 / ||y*||^2, and dL/dy."""
    S = y.shape[0]
    d = y - ystar
    den = np.sum(ystar**2, axis=(1, 2, 3))
    L = np.mean(np.sum(d**2, axis=(1, 2, 3)) / den)
    return L, 2.0 * d / (S * den[:, None, None, None])


def adam_step(p, g, m1, m2, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba, Algorithm 1) of the flat vectors; t >= 1."""
    m1 = beta1 * m1 + (1 - beta1) * g
    m2 = beta2 * m2 + (1 - beta2) * g * g
    mhat = m1 / (1 - beta1**t)
    vhat = m2 / (1 - beta2**t)
    return p - lr * mhat / (np.sqrt(vhat) + eps), m1, m2


def make_inputs(m, uI, r):
    """Network input x [5][n][n] for one medium, incident field and residual,
    and the residual scale s = ||r||_2 / n."""
    n = m.shape[0]
    s = np.linalg.norm(r) / n
    x = np.stack([m, uI.real, uI.imag, r.real / s, r.imag / s])
    return x, s


def apply(params, m, uI, r, modes=MODES, layers=LAYERS):
    """z = r + s (y_0 + i y_1): the network as a map from a residual r to an
    approximation of H^{-1} r."""
    x, s = make_inputs(m, uI, r)
    y, _ = forward(params, x[None], modes, layers)
    return r + s * (y[0, 0] + 1j * y[0, 1])
