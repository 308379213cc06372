"""Seeded synthetic inputs shared by the tests, the smoke check and the
benchmark.  Holds no arithmetic of the method itself: velocity models, source
positions, random vectors and request streams only.

The velocity models stand in for the paper's benchmark models (Sec. 3: the
homogeneous and linear-gradient media, and the SEG/EAGE overthrust / salt and
GO_3D_OBS models, whose data are not used here): same G ranges, contrasts and
grid shapes, synthetic content.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "homogeneous", "gradient_z", "random_field_model", "smooth_random_model", "surface_sources",
    "random_vectors", "serving_requests", "WORKLOADS",
]


def homogeneous(dims, c=2000.0):
    """Constant velocity, array [nz, ny, nx] float32."""
    nx, ny, nz = dims
    return np.full((nz, ny, nx), c, dtype=np.float32)


def gradient_z(dims, h, c0=1500.0, a=0.7):
    """c(z) = c0 + a z with z = k h (a vertical linear gradient)."""
    nx, ny, nz = dims
    z = np.arange(nz, dtype=np.float64) * h
    col = (c0 + a * z).astype(np.float32)
    return np.broadcast_to(col[:, None, None], (nz, ny, nx)).copy()


def random_field_model(dims, h, seed, c_top=1500.0, c_bottom=4500.0, std=300.0,
                       corr=500.0, n_planes=4, jump=(1.2, 1.4), body_c=3500.0,
                       body_axes=(1000.0, 750.0, 400.0), clip=(1500.0, 6500.0)):
    """Heterogeneous sharp-contrast model: background increasing linearly with
    depth, a smooth Gaussian random field (white noise smoothed by
    exp(-r^2 / corr^2), rescaled to ``std``), ``n_planes`` dipping planes that
    multiply the velocity below them by U(jump), one ellipsoidal body of
    ``body_c`` at the centre (semi-axes at most a quarter of the extent),
    clipped.  float32 [nz, ny, nx]."""
    nx, ny, nz = dims
    rng = np.random.Generator(np.random.PCG64(seed))
    z = np.arange(nz) * h
    y = np.arange(ny) * h
    x = np.arange(nx) * h
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    zmax = max(z[-1], h)
    c = c_top + (c_bottom - c_top) * Z / zmax
    # Gaussian random field through FFT smoothing (periodic, then rescaled)
    noise = rng.standard_normal((nz, ny, nx))
    kz = np.fft.fftfreq(nz, d=h) * 2 * np.pi
    ky = np.fft.fftfreq(ny, d=h) * 2 * np.pi
    kx = np.fft.rfftfreq(nx, d=h) * 2 * np.pi
    KZ, KY, KX = np.meshgrid(kz, ky, kx, indexing="ij")
    # Fourier transform of exp(-r^2/corr^2) is proportional to exp(-k^2 corr^2 / 4)
    filt = np.exp(-(KZ ** 2 + KY ** 2 + KX ** 2) * corr ** 2 / 4.0)
    field = np.fft.irfftn(np.fft.rfftn(noise) * filt, s=(nz, ny, nx), axes=(0, 1, 2))
    sd = field.std()
    if sd > 0:
        field = field / sd * std
    c = c + field
    # dipping planes: n . (p - p0) > 0 below the plane
    for _ in range(n_planes):
        dip = np.deg2rad(rng.uniform(0.0, 20.0))
        az = rng.uniform(0.0, 2 * np.pi)
        depth = rng.uniform(0.15, 0.85) * zmax
        nvec = np.array([np.sin(dip) * np.cos(az), np.sin(dip) * np.sin(az), np.cos(dip)])
        x0, y0 = x[-1] / 2, y[-1] / 2
        s = nvec[0] * (X - x0) + nvec[1] * (Y - y0) + nvec[2] * (Z - depth)
        c = np.where(s > 0, c * rng.uniform(*jump), c)
    # ellipsoidal body; its semi-axes are capped at a quarter of the model's
    # extent so that small grids keep their background (the 1000 x 750 x 400 m
    # body of the paper-sized grids would fill them)
    cx, cy, cz = x[-1] / 2, y[-1] / 2, z[-1] / 2
    ax, ay, az_ = (min(b, 0.25 * max(e, h)) for b, e in zip(body_axes, (x[-1], y[-1], z[-1])))
    inside = ((X - cx) / ax) ** 2 + ((Y - cy) / ay) ** 2 + ((Z - cz) / az_) ** 2 <= 1.0
    c = np.where(inside, body_c, c)
    return np.clip(c, *clip).astype(np.float32)


def smooth_random_model(dims, h, seed, c_range=(1600.0, 2800.0), corr=None):
    """A small heterogeneous model whose velocity spans ``c_range`` exactly:
    white noise (PCG64) smoothed by exp(-r^2 / corr^2) (corr = 3 h by
    default), mapped linearly onto the range.  For grids too small for the
    random-field model, whose interfaces and body saturate them.  float32
    [nz, ny, nx]."""
    nx, ny, nz = dims
    corr = 3.0 * h if corr is None else corr
    rng = np.random.Generator(np.random.PCG64(seed))
    noise = rng.standard_normal((nz, ny, nx))
    kz = np.fft.fftfreq(nz, d=h) * 2 * np.pi
    ky = np.fft.fftfreq(ny, d=h) * 2 * np.pi
    kx = np.fft.rfftfreq(nx, d=h) * 2 * np.pi
    KZ, KY, KX = np.meshgrid(kz, ky, kx, indexing="ij")
    filt = np.exp(-(KZ ** 2 + KY ** 2 + KX ** 2) * corr ** 2 / 4.0)
    field = np.fft.irfftn(np.fft.rfftn(noise) * filt, s=(nz, ny, nx), axes=(0, 1, 2))
    lo, hi = c_range
    span = field.max() - field.min()
    t = (field - field.min()) / span if span > 0 else np.zeros_like(field)
    return (lo + (hi - lo) * t).astype(np.float32)


def surface_sources(dims, nsrc, depth_index, margin):
    """``nsrc`` node positions (i, j, k) evenly spaced along x at the y centre,
    at z index ``depth_index``, x in [margin, nx - 1 - margin]."""
    nx, ny, nz = dims
    if nsrc == 1:
        xs = [nx // 2]
    else:
        xs = np.round(np.linspace(margin, nx - 1 - margin, nsrc)).astype(int).tolist()
    return [(int(i), ny // 2, int(depth_index)) for i in xs]


def random_vectors(n, nrhs, seed, dtype=np.complex128):
    """nrhs complex vectors of length n, [nrhs, n], standard normal parts."""
    rng = np.random.Generator(np.random.PCG64(seed))
    v = rng.standard_normal((nrhs, n)) + 1j * rng.standard_normal((nrhs, n))
    return v.astype(dtype)


def serving_requests(n_req, seed, rate_hz, freq_range=(2.5, 10.0),
                     dims_choices=((64, 64, 64), (96, 96, 96), (128, 128, 128),
                                   (192, 192, 96), (256, 256, 128)),
                     nrhs_max=128, min_g=4.0, c_min=1500.0):
    """A Poisson stream of solve requests: arrival time, model seed, frequency,
    grid dims, grid step h = c_min / (min_g f) (so the smallest G is min_g) and
    the number of right-hand sides (log-uniform in 1..nrhs_max)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t = 0.0
    out = []
    for r in range(n_req):
        t += rng.exponential(1.0 / rate_hz)
        f = float(rng.uniform(*freq_range))
        dims = tuple(int(d) for d in dims_choices[rng.integers(len(dims_choices))])
        nrhs = int(np.clip(np.round(np.exp(rng.uniform(0.0, np.log(nrhs_max)))), 1, nrhs_max))
        out.append({"id": r, "t_arrival": t, "model_seed": int(rng.integers(1 << 31)),
                    "freq": f, "dims": dims, "h": c_min / (min_g * f), "nrhs": nrhs})
    return out


# Named workloads: shapes of the benchmark configurations.
WORKLOADS = {
    "homog41": dict(dims=(41, 41, 41), h=20.0, freq=10.0, npml=8, kind="homogeneous",
                    c=2000.0, src=[(20, 20, 20)]),
    "gradz101": dict(dims=(101, 101, 101), h=25.0, freq=5.0, npml=10, kind="gradient",
                     c0=1500.0, a=0.7, src=[(50, 50, 11)]),
    "rf201": dict(dims=(201, 201, 101), h=25.0, freq=(4.0, 6.0, 8.0), npml=8,
                  kind="random_field", nsrc=64, src_depth=9),
    "rf400": dict(dims=(400, 400, 200), h=25.0, freq=10.0, npml=8, kind="random_field",
                  nsrc=16, src_depth=9),
}
