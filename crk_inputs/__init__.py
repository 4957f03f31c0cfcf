"""Seeded synthetic particle sets for the CRKSPH neighbour passes.

This module only draws inputs: positions, support radii, masses and gas
states. It holds none of the method's arithmetic, so both the GPU library
and the FP64 oracle can be fed from it without sharing any computation.

Every generator is driven by numpy's Philox counter-based generator keyed by
(seed, box), so a box can be regenerated bit-identically on its own (the
paper draws its initial-condition noise from a counter-based generator for
the same reason, Sec. 3.5).

Conventions shared by every generator:
  * a periodic cube of side L (default 1) holds the particles;
  * ``H`` is the kernel support radius (the paper's h in eq. C4: W = 0 for
    |x| >= h); the "h" of the workload descriptions is H/2;
  * velocities are returned component-major, shape (3, N).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "ParticleSet", "philox", "lattice_box", "lognormal_box", "clustered_clump_box",
    "batch_boxes", "support_for_neighbours", "hnet_init", "sod_tube",
]


def philox(seed: int, box: int = 0) -> np.random.Generator:
    """Counter-based generator keyed by (seed, box)."""
    key = np.array([seed & 0xFFFFFFFFFFFFFFFF, box & 0xFFFFFFFFFFFFFFFF], dtype=np.uint64)
    return np.random.Generator(np.random.Philox(key=key))


def support_for_neighbours(nngb: float, number_density: np.ndarray | float) -> np.ndarray:
    """Support radius whose sphere holds ``nngb`` particles at the given number density.

    This is only the input recipe (a sphere of radius H at density n holds
    (4 pi / 3) H^3 n particles); the library never calls it.
    """
    return np.cbrt(3.0 * nngb / (4.0 * math.pi * np.asarray(number_density, dtype=np.float64)))


@dataclass
class ParticleSet:
    """One periodic box of gas particles (all float64, original order)."""
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    H: np.ndarray
    m: np.ndarray
    u: np.ndarray
    v: np.ndarray                # (3, N)
    rho: np.ndarray | None       # None: density is m / V
    L: float = 1.0
    gamma: float = 5.0 / 3.0
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    def pos(self) -> np.ndarray:
        return np.stack([self.x, self.y, self.z])


def _wrap(a: np.ndarray, L: float) -> np.ndarray:
    a = np.mod(a, L)
    a[a >= L] -= L          # np.mod can return L for tiny negative inputs
    return a


def lattice_box(n_side: int = 32, seed: int = 1, box: int = 0, jitter: float = 0.1,
                nngb: float = 64.0, L: float = 1.0, rho0: float = 1.0, u0: float = 1.0,
                vamp: float = 0.01, gamma: float = 5.0 / 3.0) -> ParticleSet:
    """Jittered cubic lattice with a uniform gas state.

    Particle (ix, iy, iz) sits at ((i + 1/2) + U(-jitter, jitter)) * L / n_side per
    coordinate, wrapped into [0, L). Index order is ix fastest. Masses give
    density ``rho0``; the density is also passed explicitly. The flow is a
    shear v_x = vamp * sin(2 pi y / L). H is uniform, sized for ``nngb``
    particles inside the support at the mean number density.
    """
    g = philox(seed, box)
    n = n_side ** 3
    iz, iy, ix = np.meshgrid(np.arange(n_side), np.arange(n_side), np.arange(n_side), indexing="ij")
    base = np.stack([ix.ravel(), iy.ravel(), iz.ravel()]).astype(np.float64) + 0.5
    jit = g.uniform(-jitter, jitter, size=(3, n))
    p = _wrap((base + jit) * (L / n_side), L)
    H = np.full(n, float(support_for_neighbours(nngb, n / L ** 3)) )
    m = np.full(n, rho0 * L ** 3 / n)
    v = np.zeros((3, n))
    v[0] = vamp * np.sin(2.0 * math.pi * p[1] / L)
    return ParticleSet(p[0].copy(), p[1].copy(), p[2].copy(), H, m, np.full(n, u0), v,
                       np.full(n, rho0), L=L, gamma=gamma,
                       meta=dict(kind="lattice", n_side=n_side, seed=seed, box=box, jitter=jitter,
                                 nngb=nngb))


def gaussian_field(n_grid: int, spectral_index: float, g: np.random.Generator) -> np.ndarray:
    """Unit-variance Gaussian random field on an n^3 periodic grid with P(k) ~ k^n.

    White noise is filtered in Fourier space by sqrt(P(k)) (k in grid units,
    the k = 0 mode removed), then standardised.
    """
    w = g.standard_normal((n_grid, n_grid, n_grid))
    wk = np.fft.rfftn(w)
    kx = np.fft.fftfreq(n_grid) * n_grid
    kz = np.fft.rfftfreq(n_grid) * n_grid
    k2 = kx[:, None, None] ** 2 + kx[None, :, None] ** 2 + kz[None, None, :] ** 2
    amp = np.zeros_like(k2)
    nz = k2 > 0
    amp[nz] = k2[nz] ** (spectral_index / 4.0)       # sqrt(k^n) = (k^2)^(n/4)
    f = np.fft.irfftn(wk * amp, s=w.shape, axes=(0, 1, 2))
    f -= f.mean()
    f /= f.std()
    return f


def smooth_field(f: np.ndarray, width: float) -> np.ndarray:
    """Periodic Gaussian smoothing of a grid field, width in grid cells."""
    n = f.shape[0]
    k = np.fft.fftfreq(n) * 2.0 * math.pi
    kz = np.fft.rfftfreq(n) * 2.0 * math.pi
    k2 = k[:, None, None] ** 2 + k[None, :, None] ** 2 + kz[None, None, :] ** 2
    return np.fft.irfftn(np.fft.rfftn(f) * np.exp(-0.5 * k2 * width * width), s=f.shape,
                         axes=(0, 1, 2))


def lognormal_box(n_side: int = 128, sigma: float = 1.5, spectral_index: float = -2.0,
                  seed: int = 2, box: int = 0, nngb: float = 64.0, L: float = 1.0,
                  n_grid: int | None = None, n_particles: int | None = None,
                  u0: float = 1.0, vamp: float = 0.01, vnoise: float = 0.01,
                  hcap: float = 0.3, rho_input: float | None = None,
                  gamma: float = 5.0 / 3.0, h_smooth: float = 1.0) -> ParticleSet:
    """Lognormal clustered particle set.

    A Gaussian field g with P(k) ~ k^spectral_index on an n_grid^3 grid gives the
    cell density rho_c = exp(sigma g - sigma^2/2), normalised to mean 1. Cell
    occupancies are multinomial over cells with probabilities ~ rho_c, and each
    particle is uniform inside its cell. Particles are stored cell by cell in
    grid order (x fastest). H_i puts ``nngb`` particles in the support at the
    density of its cell after a Gaussian smoothing of rho_c over ``h_smooth``
    grid cells (0: no smoothing), clamped to ``hcap * L`` (the clamp count is
    in meta). Without the smoothing a support sized from one cell's density
    can hold from 2 to ~10^4 particles, because the field is rough at the grid
    scale; one cell of smoothing gives the ~20-400 range of the workload.
    Velocities: shear v_x = vamp sin(2 pi y / L) plus N(0, vnoise^2) per
    component. Masses are equal, total mass L^3 (mean density 1); when
    ``rho_input`` is None the density is left to the library (m / V).
    """
    g = philox(seed, box)
    n_grid = n_grid or n_side
    N = n_particles or n_side ** 3
    field_ = gaussian_field(n_grid, spectral_index, g)
    rho_c = np.exp(sigma * field_ - 0.5 * sigma * sigma)
    rho_c /= rho_c.mean()
    flat = rho_c.ravel()                       # index = (iz * n + iy) * n + ix
    counts = g.multinomial(N, flat / flat.sum())
    cell = np.repeat(np.arange(flat.size), counts)
    ix = cell % n_grid
    iy = (cell // n_grid) % n_grid
    iz = cell // (n_grid * n_grid)
    off = g.uniform(0.0, 1.0, size=(3, N))
    h = L / n_grid
    p = _wrap(np.stack([ix + off[0], iy + off[1], iz + off[2]]) * h, L)
    rho_h = smooth_field(rho_c, h_smooth).ravel() if h_smooth > 0 else flat
    rho_h = np.maximum(rho_h, 1e-12)
    H = support_for_neighbours(nngb, N * rho_h[cell] / L ** 3)
    nclamp = int(np.count_nonzero(H > hcap * L))
    H = np.minimum(H, hcap * L)
    v = g.normal(0.0, vnoise, size=(3, N))
    v[0] += vamp * np.sin(2.0 * math.pi * p[1] / L)
    m = np.full(N, L ** 3 / N)
    rho = None if rho_input is None else np.full(N, rho_input)
    return ParticleSet(p[0].copy(), p[1].copy(), p[2].copy(), H, m, np.full(N, u0), v, rho,
                       L=L, gamma=gamma,
                       meta=dict(kind="lognormal", n_side=n_side, n_grid=n_grid, sigma=sigma,
                                 spectral_index=spectral_index, seed=seed, box=box, nngb=nngb,
                                 n_clamped=nclamp, hcap=hcap, h_smooth=h_smooth))


def clustered_clump_box(n_side: int = 256, sigma: float = 2.0, spectral_index: float = -2.5,
                        seed: int = 5, n_clumps: int = 64, clump_frac: float = 0.01,
                        overdensity: float = 100.0, nngb: float = 64.0, L: float = 1.0,
                        hcap: float = 0.3) -> ParticleSet:
    """Lognormal field plus dense uniform spheres.

    (1 - clump_frac) of the n_side^3 particles follow ``lognormal_box``; the
    rest are split evenly over ``n_clumps`` uniform spheres at ``overdensity``
    times the mean density, centred on the densest grid cells. Clump
    particles get H sized for ``nngb`` neighbours at the clump density.
    """
    N = n_side ** 3
    per = int(N * clump_frac) // n_clumps
    n_clump_tot = per * n_clumps
    base = lognormal_box(n_side=n_side, sigma=sigma, spectral_index=spectral_index, seed=seed,
                         nngb=nngb, L=L, n_particles=N - n_clump_tot, hcap=hcap)
    g = philox(seed, 1)
    field_ = gaussian_field(n_side, spectral_index, philox(seed, 0))
    order = np.argsort(field_.ravel())[::-1][:n_clumps]
    cz, cy, cx = np.unravel_index(order, field_.shape)
    centres = (np.stack([cx, cy, cz]).astype(np.float64) + 0.5) * (L / n_side)
    R = float(np.cbrt(3.0 * per / (4.0 * math.pi * overdensity * N / L ** 3)))
    # uniform points in a ball: direction from normalised Gaussians, radius R u^(1/3)
    dirs = g.standard_normal((3, n_clump_tot))
    dirs /= np.linalg.norm(dirs, axis=0)
    rad = R * np.cbrt(g.uniform(0.0, 1.0, n_clump_tot))
    pc = _wrap(np.repeat(centres, per, axis=1) + dirs * rad, L)
    Hc = np.full(n_clump_tot, float(support_for_neighbours(nngb, overdensity * N / L ** 3)))
    vc = g.normal(0.0, 0.01, size=(3, n_clump_tot))
    vc[0] += 0.01 * np.sin(2.0 * math.pi * pc[1] / L)
    meta = dict(base.meta)
    meta.update(kind="lognormal+clumps", n_side=n_side, n_clumps=n_clumps, clump_radius=R,
                n_in_clumps=n_clump_tot)
    return ParticleSet(np.concatenate([base.x, pc[0]]), np.concatenate([base.y, pc[1]]),
                       np.concatenate([base.z, pc[2]]), np.concatenate([base.H, Hc]),
                       np.full(N, L ** 3 / N), np.ones(N), np.concatenate([base.v, vc], axis=1),
                       None, L=L, meta=meta)


def batch_boxes(n_boxes: int = 512, seed: int = 3, n_min: int = 8, n_max: int = 48,
                nngb: float = 64.0, hcap: float = 0.3) -> list[ParticleSet]:
    """Independent periodic unit boxes of uneven size.

    Box b uses generator key (seed, b): side n_b = round(exp(U(ln n_min, ln n_max))),
    N_b = n_b^3; half the boxes (U < 1/2) are jittered lattices, half lognormal
    (sigma 1.5, P ~ k^-2) on an n_b^3 grid with H clamped to hcap. Each box gets
    a gamma-law gas state with rho_b, u_b log-uniform in [0.1, 10] and equal
    masses m = rho_b / N_b; the density is left to the library (m / V).
    """
    boxes = []
    for b in range(n_boxes):
        g = philox(seed, b)
        nb = int(round(math.exp(g.uniform(math.log(n_min), math.log(n_max)))))
        lattice = bool(g.uniform() < 0.5)
        rho_b = math.exp(g.uniform(math.log(0.1), math.log(10.0)))
        u_b = math.exp(g.uniform(math.log(0.1), math.log(10.0)))
        sub = 1000 + b
        if lattice:
            ps = lattice_box(n_side=nb, seed=seed, box=sub, nngb=nngb, rho0=rho_b, u0=u_b)
        else:
            ps = lognormal_box(n_side=nb, seed=seed, box=sub, nngb=nngb, u0=u_b, hcap=hcap)
        ps.m = np.full(ps.n, rho_b / ps.n)
        ps.u = np.full(ps.n, u_b)
        ps.rho = None
        ps.meta.update(rho_b=rho_b, u_b=u_b, batch_box=b)
        boxes.append(ps)
    return boxes


def hnet_init(seed: int = 0, n_in: int = 8, n_hidden: int = 64) -> np.ndarray:
    """Seeded starting weights of the 8 -> 64 -> 64 -> 1 smoothing-length network.

    Flat FP64 vector in the order W1 (n_hidden x n_in, row-major), b1,
    W2 (n_hidden x n_hidden), b2, w3 (n_hidden), b3: weights uniform in
    +-sqrt(6 / fan_in) (halved for the output row), biases zero.
    """
    g = philox(seed, 77)
    parts = []
    for name, shp, fan in (("W1", (n_hidden, n_in), n_in), ("b1", (n_hidden,), 0),
                           ("W2", (n_hidden, n_hidden), n_hidden), ("b2", (n_hidden,), 0),
                           ("w3", (n_hidden,), n_hidden), ("b3", (1,), 0)):
        if fan:
            lim = math.sqrt(6.0 / fan) * (0.5 if name == "w3" else 1.0)
            parts.append(g.uniform(-lim, lim, size=shp).ravel())
        else:
            parts.append(np.zeros(int(np.prod(shp))))
    return np.concatenate(parts)


def sod_tube(n_high: int = 20, nngb: float = 64.0, gamma: float = 5.0 / 3.0) -> ParticleSet:
    """Shock tube with two Riemann interfaces in the periodic cube [0, 2)^3.

    High state (rho = 1, P = 1) in x in [0, 0.5) and [1.5, 2), low state
    (rho = 1/8, P = 1/8) in [0.5, 1.5): the same temperature on both sides,
    so u = P / ((gamma - 1) rho) is uniform. Equal-mass particles on cubic
    lattices of spacing d = 0.5 / n_high (high) and 2 d (low), so the 3D
    density ratio is 8 and the tube is n_high + n_high/2 particles long over
    [0, 1). The interfaces are sharp (a step function); the gas is at rest.
    H holds ``nngb`` lattice neighbours of each side.
    """
    L = 2.0
    d = 0.5 / n_high
    parts = []
    for x0, x1, sp in ((0.0, 0.5, d), (0.5, 1.5, 2.0 * d), (1.5, 2.0, d)):
        nx = int(round((x1 - x0) / sp))
        ny = int(round(L / sp))
        gx = x0 + (np.arange(nx) + 0.5) * sp
        gy = (np.arange(ny) + 0.5) * sp
        X, Y, Z = np.meshgrid(gx, gy, gy, indexing="ij")
        Hs = support_for_neighbours(nngb, 1.0 / sp ** 3)
        parts.append((X.ravel(), Y.ravel(), Z.ravel(), np.full(X.size, float(Hs))))
    x, y, z, H = (np.concatenate([q[k] for q in parts]) for k in range(4))
    n = x.shape[0]
    m = np.full(n, d ** 3)
    u = np.full(n, 1.0 / (gamma - 1.0))
    v = np.zeros((3, n))
    return ParticleSet(x, y, z, H, m, u, v, None, L=L, gamma=gamma,
                       meta=dict(kind="sod", n_high=n_high, spacing=d))
