"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module only draws random numbers and lays them out; it contains none of
the gravity arithmetic, so both the oracle side and the HIP side can use it.
Every generator takes an explicit seed (``numpy.random.default_rng``) and
returns float64 arrays in row-major ``(n, 3)`` / ``(n,)`` layout, total mass 1
per system, G = 1.

The paper's own test problems (Evrard collapse, polytropes, isothermal
collapse, Zeldovich pancake, the GMC) need hydro initial conditions that are
not available; these synthetic particle sets stand in for them with the
density structures the method is exercised on: a centrally concentrated
sphere, a uniform sphere with a turbulent velocity field, a clustered field
of clumps, many independent small systems, and a periodic box with one
collapsing plane-wave mode (the pancake geometry).
"""
from __future__ import annotations

import numpy as np

PLUMMER_RMAX = 10.0


def _isotropic(rng, n):
    z = rng.uniform(-1.0, 1.0, n)
    phi = rng.uniform(0.0, 2.0 * np.pi, n)
    s = np.sqrt(1.0 - z * z)
    return np.stack([s * np.cos(phi), s * np.sin(phi), z], axis=1)


def plummer_radii(rng, n, b=1.0, rmax=PLUMMER_RMAX):
    """Radii of a Plummer sphere truncated at ``rmax`` (inverse-CDF sampling)."""
    s = rmax / b
    mu_max = s ** 3 / (1.0 + s * s) ** 1.5
    u = rng.uniform(0.0, mu_max, n)
    u = np.maximum(u, 1e-300)
    return b / np.sqrt(u ** (-2.0 / 3.0) - 1.0)


def plummer(n, seed=1, b=1.0, sigma=0.4, rmax=PLUMMER_RMAX):
    """Equal-mass Plummer sphere (M = 1, scale b) truncated at ``rmax``;
    isotropic Gaussian velocities with 1D dispersion ``sigma``."""
    rng = np.random.default_rng(seed)
    r = plummer_radii(rng, n, b, rmax)
    x = _isotropic(rng, n) * r[:, None]
    v = rng.normal(0.0, sigma, (n, 3))
    m = np.full(n, 1.0 / n)
    return x, v, m


def uniform_sphere(n, seed=2, R=1.0):
    """Equal-mass particles uniform in a sphere of radius R (no velocities)."""
    rng = np.random.default_rng(seed)
    r = R * rng.uniform(0.0, 1.0, n) ** (1.0 / 3.0)
    x = _isotropic(rng, n) * r[:, None]
    m = np.full(n, 1.0 / n)
    return x, m, rng


def grf_velocities(x, rng, grid=128, slope=-4.0, rms=1.0, box=(-1.0, 1.0)):
    """Gaussian random velocity field: three independent components with power
    spectrum P(k) ~ k^slope on a ``grid``^3 mesh over ``box``^3, k = 0 removed,
    cloud-in-cell interpolated to the particles and scaled so that the 3D rms
    speed over the particles is ``rms``."""
    lo, hi = box
    k1 = np.fft.fftfreq(grid) * grid
    kz1 = np.fft.rfftfreq(grid) * grid
    kk = np.sqrt(k1[:, None, None] ** 2 + k1[None, :, None] ** 2 + kz1[None, None, :] ** 2)
    amp = np.zeros_like(kk)
    nz = kk > 0
    amp[nz] = kk[nz] ** (slope / 2.0)
    comps = []
    for _ in range(3):
        re = rng.normal(size=kk.shape)
        im = rng.normal(size=kk.shape)
        field = np.fft.irfftn((re + 1j * im) * amp, s=(grid, grid, grid))
        comps.append(field.astype(np.float64))
    # cloud-in-cell interpolation (periodic wrap at the box edge)
    g = (x - lo) / (hi - lo) * grid - 0.5
    i0 = np.floor(g).astype(np.int64)
    fr = g - i0
    v = np.zeros((x.shape[0], 3))
    for dx in (0, 1):
        wx = fr[:, 0] if dx else 1.0 - fr[:, 0]
        ix = (i0[:, 0] + dx) % grid
        for dy in (0, 1):
            wy = fr[:, 1] if dy else 1.0 - fr[:, 1]
            iy = (i0[:, 1] + dy) % grid
            for dz in (0, 1):
                wz = fr[:, 2] if dz else 1.0 - fr[:, 2]
                iz = (i0[:, 2] + dz) % grid
                wgt = wx * wy * wz
                for c in range(3):
                    v[:, c] += wgt * comps[c][ix, iy, iz]
    v -= v.mean(axis=0)
    v *= rms / np.sqrt(np.mean(np.sum(v * v, axis=1)))
    return v


def turbulent_sphere(n, seed=2, grid=128):
    """Uniform unit sphere with a k^-4 Gaussian-random-field velocity (rms 1)."""
    x, m, rng = uniform_sphere(n, seed)
    v = grf_velocities(x, rng, grid=grid)
    return x, v, m


def clumps(n, seed=3, nclump=64):
    """``nclump`` Plummer clumps with log-normal masses (sigma_ln = 1) at
    uniform random centres in the unit box.  Clump scale
    b_c = 0.02 (nclump M_c)^(1/3), truncated at 10 b_c; isotropic Gaussian
    internal velocities with the Plummer virial 1D dispersion
    sqrt(pi M_c / (32 b_c)); equal particle masses 1/n.  Returns
    (x, v, m, clump_id)."""
    rng = np.random.default_rng(seed)
    mc = np.exp(rng.normal(0.0, 1.0, nclump))
    mc /= mc.sum()
    raw = n * mc
    nc = np.floor(raw).astype(np.int64)
    rem = n - nc.sum()
    order = np.argsort(-(raw - nc), kind="stable")
    nc[order[:rem]] += 1
    centres = rng.uniform(0.0, 1.0, (nclump, 3))
    xs, vs, ids = [], [], []
    for c in range(nclump):
        k = int(nc[c])
        if k == 0:
            continue
        mcl = k / n
        bc = 0.02 * (nclump * mcl) ** (1.0 / 3.0)
        r = plummer_radii(rng, k, bc, 10.0 * bc)
        xs.append(centres[c] + _isotropic(rng, k) * r[:, None])
        sig = np.sqrt(np.pi * mcl / (32.0 * bc))
        vs.append(rng.normal(0.0, sig, (k, 3)))
        ids.append(np.full(k, c, dtype=np.int32))
    x = np.concatenate(xs)
    v = np.concatenate(vs)
    m = np.full(n, 1.0 / n)
    return x, v, m, np.concatenate(ids)


def zeldovich_box(n_side, seed=6, box=1.0, growth=0.9, jitter=1e-3):
    """Periodic cube of side ``box`` holding an n_side^3 lattice displaced by
    one plane-wave mode along x (the Zeldovich approximation): for lattice
    points q, x = q - growth (box / 2 pi) sin(2 pi q_x / box), which first
    crosses (a caustic) at growth = 1; velocities along the displacement,
    v_x = -(box / 2 pi) sin(2 pi q_x / box).  A Gaussian jitter of
    ``jitter`` lattice spacings (rms per axis) breaks the lattice symmetry.
    Positions are returned inside [0, box); equal masses 1/n."""
    rng = np.random.default_rng(seed)
    g = (np.arange(n_side) + 0.5) * (box / n_side)
    q = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    s = np.sin(2.0 * np.pi * q[:, 0] / box) * (box / (2.0 * np.pi))
    x = q.copy()
    x[:, 0] -= growth * s
    x += rng.normal(0.0, jitter * box / n_side, x.shape)
    x = np.mod(x, box)
    v = np.zeros_like(x)
    v[:, 0] = -s
    n = len(x)
    return x, v, np.full(n, 1.0 / n)


def neighbour_lengths(x, k=32, box=None):
    """Per-particle lengths that follow the local particle spacing, as fully
    adaptive softening does: the distance to the k-th nearest neighbour
    (scipy's k-d tree; periodic images when ``box`` is given)."""
    from scipy.spatial import cKDTree
    pts = np.mod(x, box) if box else x
    tree = cKDTree(pts, boxsize=box)
    d, _ = tree.query(pts, k=k + 1)
    return np.ascontiguousarray(d[:, k])


def batched_plummer(nsys=256, seed=4, nmin=1024, nmax=65536, sigma=0.4):
    """``nsys`` independent Plummer systems (each M = 1, b = 1, r <= 10) with
    sizes log-uniform in [nmin, nmax] and active fractions uniform in
    [0.01, 1].  Returns dict with x, v, m (concatenated), offsets (nsys+1),
    active (global indices, sorted within each system) and act_offsets."""
    rng = np.random.default_rng(seed)
    sizes = np.rint(np.exp(rng.uniform(np.log(nmin), np.log(nmax), nsys))).astype(np.int64)
    frac = rng.uniform(0.01, 1.0, nsys)
    xs, vs, ms, acts = [], [], [], []
    off = np.zeros(nsys + 1, dtype=np.int64)
    aoff = np.zeros(nsys + 1, dtype=np.int64)
    for s in range(nsys):
        k = int(sizes[s])
        r = plummer_radii(rng, k)
        xs.append(_isotropic(rng, k) * r[:, None])
        vs.append(rng.normal(0.0, sigma, (k, 3)))
        ms.append(np.full(k, 1.0 / k))
        na = max(1, int(round(frac[s] * k)))
        a = np.sort(rng.choice(k, size=na, replace=False)) + off[s]
        acts.append(a)
        off[s + 1] = off[s] + k
        aoff[s + 1] = aoff[s] + na
    return {"x": np.concatenate(xs), "v": np.concatenate(vs), "m": np.concatenate(ms),
            "offsets": off, "active": np.concatenate(acts).astype(np.int64),
            "act_offsets": aoff, "sizes": sizes, "frac": frac}


def adjoint_weights(n, seed=5):
    """Gaussian weights w_i ~ N(0, I_3) for L = sum_i w_i . a_i."""
    rng = np.random.default_rng(seed + 1000)
    return rng.normal(0.0, 1.0, (n, 3))


def random_subset(n, frac, seed):
    """Sorted random subset of range(n) of size max(1, round(frac n))."""
    rng = np.random.default_rng(seed)
    k = max(1, int(round(frac * n)))
    return np.sort(rng.choice(n, size=k, replace=False)).astype(np.int64)
