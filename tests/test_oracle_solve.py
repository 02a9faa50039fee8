"""Pins for the oracle's spectral integration (Sec. III-B: forward 3D FFT of
each component, integration filter j w / |w|^2, inverse 3D FFT, sum of the
components).

The closed forms use band-limited trigonometric potentials: for V = grad(phi)
the filter returns -phi (minus its mean) exactly up to rounding, on any grid,
anisotropic boxes included.  A brute-force O(n^2) DFT on tiny grids pins the
transform's axis order, sign and normalisation independently of numpy.fft.
"""
import itertools

import numpy as np
import pytest

import oracle


def _centres(dims, bbox):
    b = np.asarray(bbox, np.float32).astype(np.float64)
    h = (b[3:] - b[:3]) / np.asarray(dims)
    xs = [b[a] + (np.arange(dims[a]) + 0.5) * h[a] for a in range(3)]
    Z, Y, X = np.meshgrid(xs[2], xs[1], xs[0], indexing="ij")
    return X, Y, Z, b[3:] - b[:3]


@pytest.mark.parametrize("dims,bbox", [
    ((16, 16, 16), (-1, -1, -1, 1, 1, 1)),
    ((12, 20, 10), (-0.3, -1.0, -0.25, 0.9, 1.5, 0.75)),
    ((32, 64, 32), (-1, -2, -1, 1, 2, 1)),          # the paper's 2^r x 2^(r+1) x 2^r shape
    ((10, 6, 18), (0.0, 0.0, 0.0, 1.0, 0.4, 2.0)),
])
def test_gradient_of_trig_potential_integrates_to_minus_potential(dims, bbox):
    X, Y, Z, L = _centres(dims, bbox)
    rng = np.random.default_rng(sum(dims))
    phi = np.zeros(X.shape)
    gx, gy, gz = np.zeros(X.shape), np.zeros(X.shape), np.zeros(X.shape)
    for _ in range(4):
        k = [rng.integers(-(dims[a] // 2) + 1, dims[a] // 2) for a in range(3)]
        if not any(k):
            k[0] = 1
        w = [2 * np.pi * k[a] / L[a] for a in range(3)]
        ph = rng.uniform(0, 2 * np.pi)
        amp = rng.uniform(0.5, 2.0)
        arg = w[0] * X + w[1] * Y + w[2] * Z + ph
        phi += amp * np.cos(arg)
        gx += -amp * w[0] * np.sin(arg)
        gy += -amp * w[1] * np.sin(arg)
        gz += -amp * w[2] * np.sin(arg)
    A, imag = oracle.indicator(np.stack([gx, gy, gz]), dims, bbox, return_imag=True)
    expect = -(phi - phi.mean())
    scale = np.abs(phi).max()
    assert np.max(np.abs(A - expect)) < 1e-11 * scale
    assert imag < 1e-11 * scale


def test_constant_field_integrates_to_zero_and_mean_is_zero():
    dims, bbox = (8, 12, 10), (-1, -1, -1, 1, 1, 1)
    V = np.ones((3,) + dims[::-1]) * np.array([0.3, -1.2, 2.0])[:, None, None, None]
    A = oracle.indicator(V, dims, bbox)
    assert np.max(np.abs(A)) < 1e-13
    rng = np.random.default_rng(1)
    A = oracle.indicator(rng.standard_normal((3,) + dims[::-1]), dims, bbox)
    assert abs(A.mean()) < 1e-13


def test_nyquist_plane_uses_full_wavenumber_in_denominator():
    """V_y = (-1)^qx cos(2 pi (qy + 1/2) / Ny * 1 + c): the x wavenumber is the
    Nyquist one, kappa_x = -Nx/2, which still enters |w|^2."""
    dims, bbox = (8, 12, 6), (-1.0, -1.5, -0.5, 1.0, 1.5, 0.5)
    X, Y, Z, L = _centres(dims, bbox)
    qx = np.arange(dims[0])[None, None, :]
    wy = 2 * np.pi / L[1]
    c0 = 0.4
    Vy = (-1.0) ** qx * np.cos(wy * Y + c0)
    A = oracle.indicator(np.stack([np.zeros_like(Vy), Vy, np.zeros_like(Vy)]), dims, bbox)
    wx = np.pi * dims[0] / L[0]
    # derivative of cos is -w sin; the filter divides by |w|^2 = wx^2 + wy^2
    expect = (-1.0) ** qx * np.sin(wy * Y + c0) * (-wy) / (wx ** 2 + wy ** 2)
    assert np.max(np.abs(A - expect)) < 1e-12


def _brute_dft3(f, sign):
    """O(n^2) 3D DFT over array axes (z, y, x), exp(sign * 2 pi i k.q / N)."""
    nz, ny, nx = f.shape
    out = np.zeros(f.shape, complex)
    for kz, ky, kx in itertools.product(range(nz), range(ny), range(nx)):
        s = 0j
        for qz, qy, qx in itertools.product(range(nz), range(ny), range(nx)):
            ph = kz * qz / nz + ky * qy / ny + kx * qx / nx
            s += f[qz, qy, qx] * np.exp(sign * 2j * np.pi * ph)
        out[kz, ky, kx] = s
    return out


@pytest.mark.parametrize("dims", [(4, 6, 2), (2, 2, 2), (6, 4, 4)])
def test_transform_against_brute_force_dft(dims):
    """The indicator with numpy's FFT equals the same filter applied through a
    brute-force DFT (forward e^-, inverse e^+ with 1/n), on tiny grids."""
    bbox = (0, 0, 0, 1.0, 1.5, 0.5)
    rng = np.random.default_rng(11)
    V = rng.standard_normal((3,) + dims[::-1])
    dx, dy, dz, inv = oracle.filter_factors(dims, bbox)
    n = np.prod(dims)
    A = np.zeros(dims[::-1])
    for c, d in enumerate((dx, dy, dz)):
        spec = _brute_dft3(V[c], -1)
        A += (_brute_dft3(1j * d * spec * inv, +1) / n).real
    assert np.allclose(oracle.indicator(V, dims, bbox), A, rtol=1e-11, atol=1e-12)


def test_filter_frequency_units_follow_box_extent():
    """Doubling the box (same samples) doubles A: w scales as 1/L and the
    filter as 1/w."""
    dims = (8, 10, 12)
    rng = np.random.default_rng(2)
    V = rng.standard_normal((3,) + dims[::-1])
    A1 = oracle.indicator(V, dims, (0, 0, 0, 1.0, 1.2, 0.8))
    A2 = oracle.indicator(V, dims, (0, 0, 0, 2.0, 2.4, 1.6))
    assert np.allclose(A2, 2 * A1, rtol=1e-12, atol=1e-13)
