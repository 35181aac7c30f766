"""Seeded synthetic ERA5-shaped fields.

These stand in for the ERA5 reanalysis fields the paper benchmarks on (the
Benchmarks section's error-statistics set: temperature, winds, humidity on
regular latitude-longitude grids), which are not available here.  No ERA5
values are reproduced: each generator only mimics a field's spectrum and
value distribution.

This module holds no compression arithmetic; it is the only code that the
GPU path, its tests and the oracle side share.

Seeds: numpy ``Generator(PCG64(SeedSequence([cfg, var, level, idx])))``;
everything is generated in float64 and cast to float32 at the end.
Grid: latitude phi_i = 90 - i*180/(ny-1) degrees, longitude lam_j = j*360/nx.
"""
import numpy as np

VARS = ("t", "u", "v", "q")


def rng(cfg, var, level, idx):
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(cfg), int(var), int(level), int(idx)])))


def grid(ny, nx):
    phi = np.deg2rad(90.0 - np.arange(ny) * (180.0 / max(ny - 1, 1)))
    lam = np.deg2rad(np.arange(nx) * (360.0 / nx))
    return phi, lam


def t_like(ny, nx, g):
    """Temperature-like: 32 sinusoids in lon/lat with wavenumbers 1..12 and
    amplitude ~ |k|^-2, scaled to [200, 310], plus iid Gaussian noise with
    sigma = 0.5% of the range (0.55)."""
    phi, lam = grid(ny, nx)
    P, Lm = np.meshgrid(phi, lam, indexing="ij")
    f = np.zeros((ny, nx))
    for _ in range(32):
        kl = g.integers(1, 13)
        kp = g.integers(1, 13)
        th = g.uniform(0.0, 2 * np.pi)
        a = 1.0 / (kl * kl + kp * kp)
        f += a * np.cos(kl * Lm + kp * P + th)
    lo, hi = f.min(), f.max()
    f = 200.0 + (f - lo) * (110.0 / (hi - lo)) if hi > lo else np.full_like(f, 255.0)
    f += g.normal(0.0, 0.005 * 110.0, size=f.shape)
    return f


def powerlaw_field(ny, nx, g):
    """Zero-mean, unit-std field with an isotropic k^-5/3 energy spectrum:
    white noise filtered by |k|^-4/3 in the 2-D Fourier domain."""
    w = g.standard_normal((ny, nx))
    F = np.fft.rfft2(w)
    ky = np.fft.fftfreq(ny) * ny
    kx = np.fft.rfftfreq(nx) * nx
    K = np.sqrt(ky[:, None] ** 2 + kx[None, :] ** 2)
    filt = np.zeros_like(K)
    filt[K > 0] = K[K > 0] ** (-4.0 / 3.0)
    f = np.fft.irfft2(F * filt, s=(ny, nx))
    f -= f.mean()
    s = f.std()
    return f / s if s > 0 else f


def wind_like(ny, nx, g):
    """Wind-like: zero mean, k^-5/3 spectrum, std 10."""
    return 10.0 * powerlaw_field(ny, nx, g)


def humidity_like(ny, nx, g):
    """Humidity-like: lognormal (sigma 1.5) with a cos^2(latitude) taper."""
    phi, _ = grid(ny, nx)
    f = powerlaw_field(ny, nx, g)
    return 1e-3 * np.exp(1.5 * f) * (np.cos(phi)[:, None] ** 2)


def field(var, ny, nx, cfg=1, level=0, idx=0):
    """One float32 field of variable ``var`` in {'t','u','v','q'}."""
    vi = VARS.index(var)
    g = rng(cfg, vi, level, idx)
    if var == "t":
        f = t_like(ny, nx, g)
    elif var in ("u", "v"):
        f = wind_like(ny, nx, g)
    else:
        f = humidity_like(ny, nx, g)
    return np.ascontiguousarray(f, dtype=np.float32)


def plain_field(ny=181, nx=360, seed=0):
    """Plain single-field workload: one temperature-like 181x360 field."""
    g = rng(0, 0, 0, seed)
    return np.ascontiguousarray(t_like(ny, nx, g), dtype=np.float32)


def era5_stack(ny=721, nx=1440, levels=37, variables=VARS, cfg=1):
    """ERA5-shaped stack: ``levels`` x ``variables`` fields (generator)."""
    for lev in range(levels):
        for v in variables:
            yield (v, lev), field(v, ny, nx, cfg=cfg, level=lev)


BATCH_GRIDS = ((91, 180), (181, 360), (361, 720), (721, 1440))


def batch_specs(n=256, cfg=2):
    """Uneven batch: grid uniform over BATCH_GRIDS, variable uniform over
    VARS, range-relative bound log-uniform in [1e-3, 1e-1]."""
    g = rng(cfg, 99, 0, 0)
    out = []
    for i in range(n):
        ny, nx = BATCH_GRIDS[int(g.integers(0, len(BATCH_GRIDS)))]
        var = VARS[int(g.integers(0, len(VARS)))]
        eps = float(10.0 ** g.uniform(-3.0, -1.0))
        out.append((ny, nx, var, eps, i))
    return out


def batch_field(spec, cfg=2):
    ny, nx, var, eps, i = spec
    return field(var, ny, nx, cfg=cfg, level=0, idx=i)


def vortex_field(ny=1801, nx=3600, var="u", level=0, cfg=4, n_vortices=8):
    """Km-scale stress field: the variable's background plus seeded
    Rankine-profile vortices (radius 50-200 km, peak 5-15x background std,
    random sign), distance measured along great circles (R = 6371 km)."""
    base = field(var, ny, nx, cfg=cfg, level=level).astype(np.float64)
    g = rng(cfg, VARS.index(var), level, 10_000)
    phi, lam = grid(ny, nx)
    sd = base.std()
    for _ in range(n_vortices):
        p0 = np.deg2rad(g.uniform(-60.0, 60.0))
        l0 = np.deg2rad(g.uniform(0.0, 360.0))
        R = g.uniform(50.0, 200.0)
        A = g.choice([-1.0, 1.0]) * g.uniform(5.0, 15.0) * sd
        # great-circle distance (haversine), rows limited to the vortex's band
        dphi = np.deg2rad(10.0 * R / 111.0 + 1.0)
        rows = np.where(np.abs(phi - p0) <= dphi)[0]
        if rows.size == 0:
            continue
        P = phi[rows][:, None]
        h = np.sin((P - p0) / 2) ** 2 + np.cos(P) * np.cos(p0) * np.sin((lam[None, :] - l0) / 2) ** 2
        r = 2 * 6371.0 * np.arcsin(np.sqrt(np.clip(h, 0.0, 1.0)))
        prof = np.where(r <= R, A * r / R, np.where(r <= 10 * R, A * R / np.maximum(r, 1e-9), 0.0))
        base[rows] += prof
    return np.ascontiguousarray(base, dtype=np.float32)
