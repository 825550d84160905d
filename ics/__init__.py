"""Seeded synthetic initial conditions for the SPH neighbour-loop workloads.

This module only draws particles. It holds none of the method's arithmetic
(no kernel, density, force or time-integration formula): both the HIP path and
the CPU oracle receive exactly the arrays produced here.

Every workload is a periodic cube of side L=1 with equal masses m=1/N, the
adiabatic index gamma=5/3 and the smoothing-length factor eta=1.2348 (about 48
weighted neighbours).  Each generator returns a dict of float64 / float32 /
int8 numpy arrays in *original* particle order:

  x (N,3) f64   positions in [0, L)
  v (N,3) f64   velocities
  m (N,)  f32   masses
  u (N,)  f32   specific internal energies
  h (N,)  f32   initial smoothing-length guess, eta * (m / rho_model)^(1/3)
                with rho_model the density the recipe was drawn from
  bin (N,) i8   initial time-bin from a model time-step (for multi-bin recipes)

plus scalar metadata.  Seeds follow numpy PCG64 with
seed = 1807_01341 + workload index (1..5) and sub-streams spawned in a fixed
order, so every draw is reproducible on any host.
"""
from __future__ import annotations

import math

import numpy as np

ETA = 1.2348
GAMMA = 5.0 / 3.0
BASE_SEED = 1807_01341
N_BINS = 14


def _streams(index: int, n: int):
    ss = np.random.SeedSequence(BASE_SEED + index)
    return [np.random.Generator(np.random.PCG64(s)) for s in ss.spawn(n)]


def _wrap(x, L=1.0):
    x = np.mod(x, L)
    x[x >= L] -= L
    x[x < 0] = 0.0
    return x


def lattice_positions(nside: int, jitter: float, rng, L: float = 1.0):
    """Cubic lattice sites (i+1/2)*d with independent U(-jitter*d, +jitter*d)
    displacements per axis (jitter=0 gives the perfect lattice)."""
    d = L / nside
    g = (np.arange(nside, dtype=np.float64) + 0.5) * d
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    x = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    if jitter > 0:
        x += rng.uniform(-jitter * d, jitter * d, size=x.shape)
    return _wrap(x, L)


def plummer_offsets(n: int, a: float, rng, rmax_over_a: float = 10.0):
    """Plummer-sphere radii by inverse transform of the enclosed-mass fraction
    M(<r)/M = r^3/(r^2+a^2)^{3/2}, truncated at r = rmax_over_a * a, with
    isotropic directions.  Returns offsets (n,3) from the centre."""
    s = rmax_over_a
    xmax = s ** 3 / (s * s + 1.0) ** 1.5
    X = rng.uniform(0.0, xmax, size=n)
    X = np.maximum(X, 1e-300)
    r = a / np.sqrt(X ** (-2.0 / 3.0) - 1.0)
    mu = rng.uniform(-1.0, 1.0, size=n)
    phi = rng.uniform(0.0, 2.0 * math.pi, size=n)
    st = np.sqrt(1.0 - mu * mu)
    return np.stack([r * st * np.cos(phi), r * st * np.sin(phi), r * mu], axis=1)


def plummer_density(r, a: float, mass: float, rmax_over_a: float = 10.0):
    """Model density of the truncated Plummer sphere drawn above."""
    s = rmax_over_a
    frac = s ** 3 / (s * s + 1.0) ** 1.5
    rho0 = 3.0 * (mass / frac) / (4.0 * math.pi * a ** 3)
    return np.where(r < s * a, rho0 * (1.0 + (r / a) ** 2) ** -2.5, 0.0)


def _h_from_model_density(rho_model, m):
    return (ETA * np.cbrt(m / rho_model)).astype(np.float32)


def _model_bins(h_model, u, n_bins=N_BINS, courant=0.2):
    """Initial time-bins from a model time-step proportional to h/c_s,
    quantised to powers of two of the smallest one (bins 0..n_bins-1)."""
    cs = np.sqrt(GAMMA * (GAMMA - 1.0) * u.astype(np.float64))
    dt = courant * h_model.astype(np.float64) / cs
    tmin = dt.min()
    b = np.floor(np.log2(dt / tmin)).astype(np.int64)
    return np.clip(b, 0, n_bins - 1).astype(np.int8), float(tmin)


def tiny_lattice(nside: int = 16, jitter: float = 0.1, velocity_sigma: float = 0.0,
                 index: int = 1):
    """Workload 1: nside^3 jittered lattice, u=1, all particles in bin 0.
    velocity_sigma>0 draws Gaussian velocities with that standard deviation
    in units of the sound speed (the moving variant)."""
    r_pos, r_vel = _streams(index, 2)
    N = nside ** 3
    x = lattice_positions(nside, jitter, r_pos)
    u = np.ones(N, np.float32)
    m = np.full(N, 1.0 / N, np.float32)
    v = np.zeros((N, 3))
    if velocity_sigma > 0:
        cs = math.sqrt(GAMMA * (GAMMA - 1.0) * 1.0)
        v = r_vel.normal(0.0, velocity_sigma * cs, size=(N, 3))
    h = np.full(N, ETA / nside, np.float32)
    return dict(x=x, v=v, m=m, u=u, h=h, bin=np.zeros(N, np.int8), L=1.0, name=f"lattice{nside}^3")


def perfect_lattice(nside: int):
    """Unjittered lattice with m = d^3 (mean density 1), u = 1, v = 0."""
    x = lattice_positions(nside, 0.0, None)
    N = nside ** 3
    return dict(x=x, v=np.zeros((N, 3)), m=np.full(N, 1.0 / N, np.float32),
                u=np.ones(N, np.float32), h=np.full(N, ETA / nside, np.float32),
                bin=np.zeros(N, np.int8), L=1.0, name=f"perfect{nside}^3")


def clustered(n_total: int = 2_097_152, n_clumps: int = 20, clump_fraction: float = 0.1,
              a_range=(0.002, 0.02), u_range=(1e-2, 1e2), index: int = 2):
    """Workload 2: uniform random background plus Plummer spheres with seeded
    centres and log-uniform scale radii, u log-uniform, model time-bins."""
    r_bg, r_cen, r_a, r_cl, r_u = _streams(index, 5)
    n_cl_tot = int(round(clump_fraction * n_total))
    n_bg = n_total - n_cl_tot
    xs = [r_bg.uniform(0.0, 1.0, size=(n_bg, 3))]
    m = 1.0 / n_total
    rho_model = [np.full(n_bg, n_bg * m)]
    centres = r_cen.uniform(0.0, 1.0, size=(n_clumps, 3))
    a_s = np.exp(r_a.uniform(math.log(a_range[0]), math.log(a_range[1]), size=n_clumps))
    base, rem = divmod(n_cl_tot, n_clumps)
    for k in range(n_clumps):
        nk = base + (1 if k < rem else 0)
        off = plummer_offsets(nk, a_s[k], r_cl)
        xs.append(centres[k] + off)
        rho_model.append(plummer_density(np.linalg.norm(off, axis=1), a_s[k], nk * m)
                         + n_bg * m)
    x = _wrap(np.concatenate(xs, axis=0))
    rho_model = np.concatenate(rho_model)
    N = x.shape[0]
    u = np.exp(r_u.uniform(math.log(u_range[0]), math.log(u_range[1]), size=N)).astype(np.float32)
    mm = np.full(N, m, np.float32)
    h = _h_from_model_density(rho_model, m)
    b, tmin = _model_bins(h, u)
    return dict(x=x, v=np.zeros((N, 3)), m=mm, u=u, h=h, bin=b, t_min_model=tmin,
                L=1.0, clump_centres=centres, clump_a=a_s, name=f"clustered{N}")


def lattice_plus_clump(n_lattice_side: int, n_clump: int, a: float, rng_pos, rng_cl,
                       centre=None, jitter=0.1):
    """A jittered lattice plus one Plummer clump (both in the unit box)."""
    x_lat = lattice_positions(n_lattice_side, jitter, rng_pos)
    N = x_lat.shape[0] + n_clump
    m = 1.0 / N
    if centre is None:
        centre = rng_cl.uniform(0.0, 1.0, size=3)
    off = plummer_offsets(n_clump, a, rng_cl)
    x = _wrap(np.concatenate([x_lat, centre + off], axis=0))
    rho_bg = x_lat.shape[0] * m
    rho_model = np.concatenate([np.full(x_lat.shape[0], rho_bg),
                                plummer_density(np.linalg.norm(off, axis=1), a, n_clump * m) + rho_bg])
    return x, m, rho_model


def differentiation(index: int = 4, velocity_sigma: float = 0.1):
    """Workload 4: 31^3 = 29791 jittered lattice + a 2977-particle Plummer clump
    (a = 0.01), 32768 particles, all active, Gaussian velocities with
    sigma = velocity_sigma * c_s, and a seeded Gaussian loss weight w (N,3)."""
    r_pos, r_cl, r_vel, r_w = _streams(index, 4)
    x, m, rho_model = lattice_plus_clump(31, 32768 - 31 ** 3, 0.01, r_pos, r_cl)
    N = x.shape[0]
    u = np.ones(N, np.float32)
    cs = math.sqrt(GAMMA * (GAMMA - 1.0))
    v = r_vel.normal(0.0, velocity_sigma * cs, size=(N, 3))
    w = r_w.normal(0.0, 1.0, size=(N, 3))
    return dict(x=x, v=v, m=np.full(N, m, np.float32), u=u,
                h=_h_from_model_density(rho_model, m), bin=np.zeros(N, np.int8),
                w=w, L=1.0, name="lattice31^3+clump")


def batch_of_boxes(n_boxes: int = 64, n_range=(1_000, 200_000), index: int = 3,
                   frac_range=(0.005, 1.0)):
    """Workload 3: n_boxes independent unit boxes.  Box b draws N_b log-uniform
    in n_range; it is a k_b^3 jittered lattice (k_b = floor((0.9 N_b)^{1/3}))
    plus one Plummer clump of N_b - k_b^3 particles (a = 0.01), u log-uniform
    in [1e-2, 1e2], model time-bins, and a target active fraction f_b
    log-uniform in frac_range."""
    r_n, r_f, r_seed = _streams(index, 3)
    Ns = np.round(np.exp(r_n.uniform(math.log(n_range[0]), math.log(n_range[1]), size=n_boxes))).astype(int)
    fracs = np.exp(r_f.uniform(math.log(frac_range[0]), math.log(frac_range[1]), size=n_boxes))
    seeds = r_seed.integers(0, 2 ** 31 - 1, size=n_boxes)
    boxes = []
    for b in range(n_boxes):
        g = [np.random.Generator(np.random.PCG64(s))
             for s in np.random.SeedSequence(int(seeds[b])).spawn(3)]
        k = int(math.floor((0.9 * Ns[b]) ** (1.0 / 3.0)))
        x, m, rho_model = lattice_plus_clump(k, int(Ns[b]) - k ** 3, 0.01, g[0], g[1])
        N = x.shape[0]
        u = np.exp(g[2].uniform(math.log(1e-2), math.log(1e2), size=N)).astype(np.float32)
        h = _h_from_model_density(rho_model, m)
        bins, tmin = _model_bins(h, u)
        boxes.append(dict(x=x, v=np.zeros((N, 3)), m=np.full(N, m, np.float32), u=u, h=h,
                          bin=bins, target_active_fraction=float(fracs[b]), L=1.0))
    return boxes


def _smooth_gaussian_field(n: int, length: float, rng):
    """A unit-variance Gaussian random field on the n^3 grid, white noise
    smoothed with a Gaussian of `length` grid spacings (periodic)."""
    k1 = np.fft.fftfreq(n) * 2.0 * math.pi
    kz1 = np.fft.rfftfreq(n) * 2.0 * math.pi
    KX, KY, KZ = np.meshgrid(k1, k1, kz1, indexing="ij")
    filt = np.exp(-0.5 * (KX * KX + KY * KY + KZ * KZ) * length * length)
    del KX, KY, KZ
    g = np.fft.irfftn(np.fft.rfftn(rng.normal(size=(n, n, n))) * filt, s=(n, n, n), axes=(0, 1, 2))
    return g / g.std()


def _cic_density(x, n):
    """Cloud-in-cell count of the particles on the n^3 grid (mean 1 per cell),
    and the same field read back at each particle."""
    d = 1.0 / n
    gi = x / d - 0.5
    i0 = np.floor(gi).astype(np.int64)
    f = gi - i0
    rho = np.zeros((n, n, n))
    corners = []
    for dx in (0, 1):
        wx = f[:, 0] if dx else 1 - f[:, 0]
        for dy in (0, 1):
            wy = f[:, 1] if dy else 1 - f[:, 1]
            for dz in (0, 1):
                wz = f[:, 2] if dz else 1 - f[:, 2]
                idx = ((i0[:, 0] + dx) % n, (i0[:, 1] + dy) % n, (i0[:, 2] + dz) % n)
                w = wx * wy * wz
                np.add.at(rho, idx, w)
                corners.append((idx, w))
    rho *= n ** 3 / x.shape[0]
    rho_p = np.zeros(x.shape[0])
    for idx, w in corners:
        rho_p += w * rho[idx]
    return rho, rho_p


def grf_zeldovich(nside: int = 256, spectral_index: float = -2.5, amplitude: float = 12.0,
                  index: int = 5, n_clumps: int = 16, clump_fraction: float = 0.02,
                  clump_a=(0.002, 0.01), u_scatter: float = 0.5, scatter_length: float = 8.0,
                  thermal: str = "adiabatic", u_range=(1e-2, 1e2)):
    """Workload 5: nside^3 particles.  A lattice displaced by the Zel'dovich
    field of a Gaussian random density field with P(k) ~ k^spectral_index
    (psi_k = i k delta_k / k^2, scaled to an rms displacement of `amplitude`
    lattice spacings; 12 gives this spectrum's largest contrast at 256^3,
    about 2e2 between the densest particles and the median), with
    clump_fraction of the particles (drawn at random) moved into n_clumps
    Plummer spheres (scale radii log-uniform in clump_a) centred on the
    densest cells of the displaced lattice, which carries the density
    contrast to about 1e4.

    Thermal state (thermal="adiabatic"): u = (rho / rho_median)^(gamma-1)
    times exp(u_scatter * g), g a unit Gaussian field smoothed over
    scatter_length spacings: hotter where denser, smooth in space, so that
    the time-steps of Eq. 1 form a hierarchy with geometrically fewer
    particles on the shorter steps.  thermal="loguniform" draws u
    independently per particle, log-uniform in u_range.  v = 0.  The model
    density for the initial h and the model bins is the cloud-in-cell
    density of the displaced lattice plus each clump's Plummer profile."""
    r_field, r_u, r_cl, r_g = _streams(index, 4)
    n = nside
    d = 1.0 / n
    k1 = np.fft.fftfreq(n, d=d) * 2.0 * math.pi
    kz1 = np.fft.rfftfreq(n, d=d) * 2.0 * math.pi
    KX, KY, KZ = np.meshgrid(k1, k1, kz1, indexing="ij")
    k2 = KX * KX + KY * KY + KZ * KZ
    k2[0, 0, 0] = 1.0
    amp = np.sqrt(k2 ** (spectral_index / 2.0))
    amp[0, 0, 0] = 0.0
    noise = r_field.normal(size=(n, n, n))
    dk = np.fft.rfftn(noise) * amp
    del noise, amp
    psi = []
    for K in (KX, KY, KZ):
        psi.append(np.fft.irfftn(1j * K * dk / k2, s=(n, n, n), axes=(0, 1, 2)).ravel())
    del dk, KX, KY, KZ, k2
    psi = np.stack(psi, axis=1)
    rms = math.sqrt(float(np.mean(np.sum(psi * psi, axis=1))))
    psi *= amplitude * d / rms
    x = lattice_positions(n, 0.0, None) + psi
    del psi
    x = _wrap(x)
    N = x.shape[0]
    m = 1.0 / N
    rho_grid, rho_p = _cic_density(x, n)
    rho_p = np.maximum(rho_p, 0.05)  # mean is 1 in particle units
    n_cl_tot = int(round(clump_fraction * N)) if n_clumps > 0 else 0
    if n_cl_tot > 0:
        # clump centres: the densest cells, each at least 0.1 from the ones before
        order = np.argsort(rho_grid.ravel())[::-1]
        centres = []
        for c in order[: 64 * n_clumps]:
            cc = (np.array(np.unravel_index(c, rho_grid.shape)) + 0.5) * d
            if all(np.max(np.abs((cc - q + 0.5) % 1.0 - 0.5)) >= 0.1 for q in centres):
                centres.append(cc)
            if len(centres) == n_clumps:
                break
        centres = np.array(centres)
        moved = np.sort(r_cl.choice(N, size=n_cl_tot, replace=False))
        a_s = np.exp(r_cl.uniform(math.log(clump_a[0]), math.log(clump_a[1]), size=len(centres)))
        base, rem = divmod(n_cl_tot, len(centres))
        start = 0
        for k in range(len(centres)):
            nk = base + (1 if k < rem else 0)
            sel = moved[start:start + nk]
            off = plummer_offsets(nk, a_s[k], r_cl)
            x[sel] = _wrap(centres[k] + off)
            rho_p[sel] = plummer_density(np.linalg.norm(off, axis=1), a_s[k], nk * m) + 1.0
            start += nk
    else:
        centres = np.zeros((0, 3))
        a_s = np.zeros(0)
    h = (ETA * d * np.cbrt(1.0 / rho_p)).astype(np.float32)
    if thermal == "adiabatic":
        g = _smooth_gaussian_field(n, scatter_length, r_g)
        gi = np.minimum((x / d).astype(np.int64), n - 1)
        gp = g[gi[:, 0], gi[:, 1], gi[:, 2]]
        del g
        u = ((rho_p / np.median(rho_p)) ** (GAMMA - 1.0) * np.exp(u_scatter * gp)).astype(np.float32)
    else:
        u = np.exp(r_u.uniform(math.log(u_range[0]), math.log(u_range[1]), size=N)).astype(np.float32)
    bins, tmin = _model_bins(h, u)
    return dict(x=x, v=np.zeros((N, 3)), m=np.full(N, m, np.float32), u=u, h=h, bin=bins,
                t_min_model=tmin, L=1.0, clump_centres=centres, clump_a=a_s, name=f"grf{nside}^3")


def deep_bin_for_fraction(bins, target_fraction: float, n_bins: int = N_BINS):
    """The bin m whose active set {bin <= m} has the fraction closest to
    target_fraction (ties to the smaller m)."""
    counts = np.bincount(bins.astype(np.int64), minlength=n_bins)
    cum = np.cumsum(counts) / max(1, bins.size)
    return int(np.argmin(np.abs(cum - target_fraction)))
