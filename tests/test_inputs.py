"""The input generators (no method arithmetic): the rotated sine-product medium of Sec. 5
(eq. sineprod)."""
import numpy as np

from paper_2410_17446_amd import inputs


def test_rotated_sine_medium_unrotated_is_the_product(monkeypatch):
    """With a zero angle the medium is n0 + dn sin(ks x) sin(ks y) sin(ks z), ks = k0 n0 / (sqrt(3) q)."""
    monkeypatch.setattr(inputs, "ROT_ANGLE", 0.0)
    N, dx, z, n0, dn, q = 32, 0.25, 0.7, 1.2, 0.025, 2.0
    n2 = inputs.rotated_sine_n2(N, dx, z, n0=n0, dn=dn, q=q)
    xs = inputs.coords(N, dx)
    X, Y = np.meshgrid(xs, xs)
    ks = 2 * np.pi * n0 / (np.sqrt(3) * q)
    n = n0 + dn * np.sin(ks * X) * np.sin(ks * Y) * np.sin(ks * z)
    assert np.allclose(n2, n * n, rtol=0, atol=1e-14)


def test_rotated_sine_medium_rotation_about_z(monkeypatch):
    """Axis-angle form for the axis e_z: x~ = x cos t - y sin t, y~ = x sin t + y cos t, z~ = z."""
    t = 0.3
    monkeypatch.setattr(inputs, "ROT_AXIS", (0.0, 0.0, 2.0))  # normalised by the generator
    monkeypatch.setattr(inputs, "ROT_ANGLE", t)
    N, dx, z, n0, dn = 32, 0.25, -0.4, 1.2, 0.025
    n2 = inputs.rotated_sine_n2(N, dx, z, n0=n0, dn=dn)
    xs = inputs.coords(N, dx)
    X, Y = np.meshgrid(xs, xs)
    ks = 2 * np.pi * n0 / np.sqrt(3)
    xt, yt = X * np.cos(t) - Y * np.sin(t), X * np.sin(t) + Y * np.cos(t)
    n = n0 + dn * np.sin(ks * xt) * np.sin(ks * yt) * np.sin(ks * z)
    assert np.allclose(n2, n * n, rtol=0, atol=1e-14)


def test_rotated_sine_medium_paper_parameters():
    """The paper's axis and angle: n stays within n0 +- dn and varies along z."""
    n0, dn = 1.2, 0.025
    a = inputs.rotated_sine_n2(64, 0.25, 0.0, n0=n0, dn=dn)
    b = inputs.rotated_sine_n2(64, 0.25, 0.25, n0=n0, dn=dn)
    assert a.min() >= (n0 - dn) ** 2 - 1e-12 and a.max() <= (n0 + dn) ** 2 + 1e-12
    assert np.abs(a - b).max() > 1e-3
