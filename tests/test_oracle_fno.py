"""Pins of the FP64 FNO reference (oracle/fno.py) against things other than
itself: closed-form values of GELU, NumPy's FFT for the truncated spectral
convolution, central finite differences for every gradient, and invariances
of the residual-to-correction map."""
import numpy as np
import pytest

from oracle import fno
import ls_inputs as li

TOY = dict(modes=4, layers=2)
TOY_ARCH = dict(width=6, modes=4, layers=2, hidden=8)


def toy_params(seed=0):
    rng = np.random.default_rng(seed)
    p = {}
    for k, shp in fno.param_shapes(**TOY_ARCH):
        p[k] = rng.standard_normal(shp) * (0.5 if k.startswith("spec") else 0.4)
    return p


def test_gelu_closed_form():
    # Phi(1) = 0.841344746068543, Phi(-1) = 1 - Phi(1), Phi(2) = 0.977249868051821
    assert fno.gelu(np.array(0.0)) == 0.0
    assert abs(fno.gelu(np.array(1.0)) - 0.8413447460685429) < 1e-15
    assert abs(fno.gelu(np.array(-1.0)) + 0.15865525393145707) < 1e-15
    assert abs(fno.gelu(np.array(2.0)) - 2 * 0.9772498680518208) < 1e-15
    assert fno.gelu_grad(np.array(0.0)) == 0.5
    x = np.linspace(-4, 4, 33)
    fd = (fno.gelu(x + 1e-6) - fno.gelu(x - 1e-6)) / 2e-6
    assert np.max(np.abs(fd - fno.gelu_grad(x))) < 1e-9


@pytest.mark.parametrize("n,modes", [(16, 4), (32, 16), (48, 16)])
def test_identity_mode_weights_are_numpy_lowpass(n, modes):
    """With R = I on every retained mode the spectral convolution is the
    low-pass filter rfft2 -> keep kx < M, |kz| band -> irfft2 (NumPy)."""
    rng = np.random.default_rng(n)
    C = 3
    v = rng.standard_normal((2, C, n, n))
    R = np.zeros((2 * modes, modes, C, C), complex)
    R[:, :, np.arange(C), np.arange(C)] = 1.0
    w, _ = fno.spectral_forward(v, R, modes)
    V = np.fft.rfft2(v, norm="forward")
    keep = np.zeros_like(V)
    keep[..., :modes, :modes] = V[..., :modes, :modes]
    keep[..., n - modes:, :modes] = V[..., n - modes:, :modes]
    ref = np.fft.irfft2(keep, s=(n, n), norm="forward")
    assert np.max(np.abs(w - ref)) < 1e-12 * np.max(np.abs(ref))


def test_out_of_band_mode_is_removed_and_in_band_mode_scaled():
    n, modes, C = 32, 4, 2
    j, i = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    R = np.zeros((2 * modes, modes, C, C), complex)
    R[:, :, np.arange(C), np.arange(C)] = 2.5
    hi = np.cos(2 * np.pi * (6 * i + 1 * j) / n)         # kx = 6 >= M
    lo = np.cos(2 * np.pi * (2 * i - 3 * j) / n)         # kx = 2, kz = -3
    v = np.stack([hi, lo])[None]
    w, _ = fno.spectral_forward(v, R, modes)
    assert np.max(np.abs(w[0, 0])) < 1e-13
    assert np.max(np.abs(w[0, 1] - 2.5 * lo)) < 1e-13


def _directional_fd(fun, p, d, eps=1e-5):
    return (fun(p + eps * d) - fun(p - eps * d)) / (2 * eps)


def test_gradients_match_central_differences():
    """dL/dtheta from backward() against central differences of the loss,
    one random direction per parameter block (FP64 toy network, n = 16)."""
    n, S = 16, 2
    rng = np.random.default_rng(1)
    x = rng.standard_normal((S, 5, n, n))
    ystar = rng.standard_normal((S, 2, n, n))
    p = toy_params()
    y, cache = fno.forward(p, x, **TOY)
    L, gy = fno.loss_rel(y, ystar)
    g = fno.backward(p, cache, gy, **TOY)
    for k, shp in fno.param_shapes(**TOY_ARCH):
        d = rng.standard_normal(shp)

        def loss_along(t):
            q = dict(p)
            q[k] = p[k] + t * d
            return fno.loss_rel(fno.forward(q, x, **TOY)[0], ystar)[0]

        fd = (loss_along(1e-5) - loss_along(-1e-5)) / 2e-5
        an = float(np.sum(g[k] * d))
        assert abs(fd - an) <= 1e-7 * max(1.0, abs(an)), (k, fd, an)


def test_input_gradient_of_spectral_layer_matches_differences():
    n, modes, C = 16, 4, 3
    rng = np.random.default_rng(2)
    v = rng.standard_normal((2, C, n, n))
    R = rng.standard_normal((2 * modes, modes, C, C)) + 1j * rng.standard_normal((2 * modes, modes, C, C))
    gw = rng.standard_normal((2, C, n, n))
    gv, _ = fno.spectral_backward(gw, fno.spectral_forward(v, R, modes)[1], R, modes)
    d = rng.standard_normal(v.shape)
    f = lambda t: np.sum(gw * fno.spectral_forward(v + t * d, R, modes)[0])
    fd = (f(1e-4) - f(-1e-4)) / 2e-4       # linear in v: exact up to rounding
    assert abs(fd - np.sum(gv * d)) < 1e-10 * max(1.0, abs(fd))


def test_adam_first_step_is_lr_times_sign():
    g = np.array([3.0, -0.5, 1e-3, 0.0])
    p = np.zeros(4)
    p1, m1, m2 = fno.adam_step(p, g, np.zeros(4), np.zeros(4), 1, lr=0.01, eps=0.0 + 1e-12)
    assert np.allclose(p1[:3], -0.01 * np.sign(g[:3]), rtol=1e-9)
    assert p1[3] == 0.0
    # second step with the same gradient moves by lr again (bias-corrected moments equal g, g^2)
    p2, _, _ = fno.adam_step(p1, g, m1, m2, 2, lr=0.01, eps=1e-12)
    assert np.allclose(p2[:3] - p1[:3], -0.01 * np.sign(g[:3]), rtol=1e-9)


def test_residual_map_identity_and_scale_equivariance():
    n = 32
    p = fno.unflatten(li.fno_initial_parameters(3), )
    m = li.gaussian_random_field_medium(n, seed=4)
    uI = li.plane_wave(n, 2 * np.pi * 3, 0.7)
    r = li.random_complex((n, n), 5)
    z1 = fno.apply(p, m, uI, r)
    z2 = fno.apply(p, m, uI, 7.5 * r)
    assert np.max(np.abs(z2 - 7.5 * z1)) < 1e-12 * np.max(np.abs(z2))
    q = dict(p)
    q["proj2_w"] = np.zeros_like(p["proj2_w"])
    q["proj2_b"] = np.zeros_like(p["proj2_b"])
    assert np.array_equal(fno.apply(q, m, uI, r), r)


def test_flat_layout_matches_input_generator():
    sizes = [s for _, _, s in li.fno_param_sizes()]
    shapes = [int(np.prod(s)) for _, s in fno.param_shapes()]
    assert sizes == shapes
    vec = li.fno_initial_parameters(0)
    assert np.array_equal(fno.flatten(fno.unflatten(vec)), vec)
