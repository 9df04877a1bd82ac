"""Seeded synthetic inputs shared by the GPU path's tests/bench and by the oracle.

This module holds geometry and random numbers only: density profiles are built
from coexistence densities and widths that the caller passes in, so none of the
two-phase method's arithmetic (equation of state, Maxwell construction, forcing,
collision) lives here.

Layout convention for every field: node index n = x + nx*(y + ny*z), float64;
velocity fields are structure-of-arrays, shape (D, N).

Random numbers come from SplitMix64 (Steele, Lea & Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014) used as a counter-based generator:
draw n of stream `seed` is mix(seed + (n + 1) * gamma), gamma = 0x9E3779B97F4A7C15.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass

import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, count: int, start: int = 0) -> np.ndarray:
    """Draws start..start+count-1 of the SplitMix64 stream `seed` (uint64)."""
    with np.errstate(over="ignore"):
        n = np.arange(start + 1, start + count + 1, dtype=np.uint64)
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + n * _GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform_pm(seed: int, count: int, amplitude: float) -> np.ndarray:
    """Uniform numbers in [-amplitude, amplitude) from 53-bit SplitMix64 mantissas."""
    out = np.empty(count, dtype=np.float64)
    block = 1 << 22                       # bounded temporaries for lattices of 10^8+ nodes
    for s in range(0, count, block):
        k = min(block, count - s)
        u = (splitmix64(seed, k, s) >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)
        out[s:s + k] = amplitude * (2.0 * u - 1.0)
    return out


def _grid(nx: int, ny: int, nz: int):
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return x.ravel().astype(np.float64), y.ravel().astype(np.float64), z.ravel().astype(np.float64)


def tanh_profile(d: np.ndarray, rho_liquid: float, rho_vapour: float, width: float) -> np.ndarray:
    """rho = mean + half-jump * tanh(2 d / width); d > 0 inside the liquid.

    With this form the maximum slope is (rho_l - rho_v)/width, so `width` equals
    the interface width (rho_l - rho_v)/max|grad rho|.
    """
    mean = 0.5 * (rho_liquid + rho_vapour)
    half = 0.5 * (rho_liquid - rho_vapour)
    return mean + half * np.tanh(2.0 * d / width)


def add_noise(rho: np.ndarray, seed: int, amplitude: float) -> np.ndarray:
    """Multiplicative noise rho * (1 + eta), eta ~ U(-amplitude, amplitude) per node."""
    if amplitude == 0.0:
        return rho.copy()
    eta = uniform_pm(seed, rho.size, amplitude)
    eta += 1.0
    eta *= rho
    return eta


def flat_slab(nx: int, ny: int, nz: int, rho_liquid: float, rho_vapour: float, width: float,
              lo: float | None = None, hi: float | None = None, axis: int = 0,
              noise: float = 0.0, seed: int = 0) -> np.ndarray:
    """Liquid slab occupying [lo, hi) along `axis` (default: the middle half), tanh walls."""
    n_axis = (nx, ny, nz)[axis]
    lo = n_axis / 4.0 if lo is None else lo
    hi = 3.0 * n_axis / 4.0 if hi is None else hi
    coords = _grid(nx, ny, nz)[axis]
    # interfaces sit half-way between nodes lo-1 | lo and hi-1 | hi
    d = np.minimum(coords - (lo - 0.5), (hi - 0.5) - coords)
    rho = tanh_profile(d, rho_liquid, rho_vapour, width)
    return add_noise(rho, seed, noise)


def drop(nx: int, ny: int, nz: int, radius: float, rho_liquid: float, rho_vapour: float,
         width: float, centre=None, noise: float = 0.0, seed: int = 0, bubble: bool = False) -> np.ndarray:
    """Circular (nz == 1) or spherical drop of the liquid in vapour (or a bubble if `bubble`)."""
    if centre is None:
        centre = ((nx - 1) / 2.0, (ny - 1) / 2.0, (nz - 1) / 2.0)
    cx, cy, cz = centre
    # squared offsets per axis, broadcast over the lattice (no full-size coordinate arrays)
    dx2 = (np.arange(nx, dtype=np.float64) - cx) ** 2
    dy2 = (np.arange(ny, dtype=np.float64) - cy) ** 2
    dz2 = (np.arange(nz, dtype=np.float64) - cz) ** 2 if nz > 1 else np.zeros(nz)
    r = np.sqrt((dx2[None, None, :] + dy2[None, :, None]) + dz2[:, None, None]).ravel()
    d = radius - r
    if bubble:
        d = -d
    rho = tanh_profile(d, rho_liquid, rho_vapour, width)
    return add_noise(rho, seed, noise)


def zero_velocity(D: int, N: int) -> np.ndarray:
    return np.zeros((D, N), dtype=np.float64)


def liquid_fraction(rho: np.ndarray, rho_liquid: float, rho_vapour: float) -> np.ndarray:
    return np.clip((rho - rho_vapour) / (rho_liquid - rho_vapour), 0.0, 1.0)


def pillar_mask(nx: int, ny: int, nz: int, pillar: int = 8, gap: int = 8, height: int = 16) -> np.ndarray:
    """Solid floor at z = 0 plus square pillars (x mod p < w, y mod p < w, 1 <= z <= height).

    Returns uint8, 1 = solid. Periodic wrap in z makes the floor a ceiling as well.
    """
    x, y, z = _grid(nx, ny, nz)
    x = x.astype(np.int64); y = y.astype(np.int64); z = z.astype(np.int64)
    period = pillar + gap
    solid = (z == 0) | (((x % period) < pillar) & ((y % period) < pillar) & (z >= 1) & (z <= height))
    return solid.astype(np.uint8)


def random_mask(nx: int, ny: int, nz: int, fraction: float, seed: int) -> np.ndarray:
    """Sparse random solid nodes (for bounce-back parity on tiny grids)."""
    u = (splitmix64(seed, nx * ny * nz) >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)
    return (u < fraction).astype(np.uint8)


def random_link_q(D: int, N: int, lo: float, hi: float, seed: int) -> np.ndarray:
    """Wall fractions uniform in [lo, hi) for every link of every node, shape (3,)*D + (N,):
    entry [c + 1][n] belongs to the link n -> n + c (only links into solid nodes matter)."""
    u = (splitmix64(seed, 3 ** D * N) >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)
    return (lo + (hi - lo) * u).reshape((3,) * D + (N,))


def sphere_obstacle(nx: int, ny: int, nz: int, centre, radius: float):
    """Solid ball (disc when nz = 1 and len(centre) = 2) of the given radius around
    centre, which must lie at least radius + 1 from every face (no periodic images).

    Returns (mask uint8 [N], link_q (3,)*D + (N,)): for a fluid node p and a link c whose
    end p + c is solid, link_q[c + 1][p] is the fraction q in (0, 1] at which the segment
    p -> p + c meets the sphere, the smaller root of |p + q c - centre| = radius.
    """
    D = len(centre)
    x, y, z = _grid(nx, ny, nz)
    pos = np.stack([x, y, z][:D]).astype(np.float64)
    s = np.asarray(centre, dtype=np.float64).reshape(D, 1)
    d = pos - s
    solid = (d * d).sum(0) <= radius * radius
    N = nx * ny * nz
    lq = np.zeros((3,) * D + (N,))
    for c in itertools.product((-1, 0, 1), repeat=D):
        if not any(c):
            continue
        cv = np.asarray(c, dtype=np.float64).reshape(D, 1)
        idx = [x.astype(np.int64), y.astype(np.int64), z.astype(np.int64)][:D]
        tgt = [(idx[a] + c[a]) % (nx, ny, nz)[a] for a in range(D)]
        flat = tgt[0] + nx * (tgt[1] + (ny * tgt[2] if D == 3 else 0))
        end = solid[flat] & ~solid
        cc = float((cv * cv).sum())
        dc = (d * cv).sum(0)
        disc = np.maximum(dc * dc - cc * ((d * d).sum(0) - radius * radius), 0.0)
        q = (-dc - np.sqrt(disc)) / cc
        lq[tuple(ci + 1 for ci in c)] = np.where(end, np.clip(q, 1e-6, 1.0), 0.0)
    return solid.astype(np.uint8), lq


def _link_fractions(along, solid: np.ndarray, dims, iters: int = 30) -> np.ndarray:
    """Wall fractions of every link from a fluid node into a solid node, by bisection of
    an implicit surface along the link, to 2^-30. along(px, py, pz, c) returns phi(t) for
    the links from nodes (px, py, pz) in direction c: phi(t) <= 0 inside the solid,
    phi(0) > 0 >= phi(1). solid: bool [N]. Returns the (3,)*D + (N,) array of
    sphere_obstacle (zero away from walls)."""
    D = len(dims)
    nx, ny, nz = (tuple(dims) + (1,))[:3]
    N = nx * ny * nz
    lq = np.zeros((3,) * D + (N,))
    s3 = solid.reshape(nz, ny, nx)
    fluid = ~s3
    for c in itertools.product((-1, 0, 1), repeat=D):
        if not any(c):
            continue
        cz = c[2] if D == 3 else 0
        ahead = np.roll(s3, (-cz, -c[1], -c[0]), axis=(0, 1, 2))       # solid at r + c
        n = np.flatnonzero(ahead & fluid)
        if n.size == 0:
            continue
        phi = along((n % nx).astype(np.float64), ((n // nx) % ny).astype(np.float64),
                    (n // (nx * ny)).astype(np.float64), (c[0], c[1], cz))
        lo = np.zeros(n.size)
        hi = np.ones(n.size)
        for _ in range(iters):
            mid = 0.5 * (lo + hi)
            inside = phi(mid) <= 0
            hi = np.where(inside, mid, hi)
            lo = np.where(inside, lo, mid)
        lq[tuple(ci + 1 for ci in c)][n] = np.clip(hi, 1e-6, 1.0)
    return lq


def tapered_posts(nx: int, ny: int, nz: int, floor: int, r_base: float, r_tip: float, height: float,
                  spacing: int):
    """Flat substrate with tapered posts in a square arrangement (the curved-wall geometry of
    drops bouncing off tapered posts), z vertical.

    The solid floor is the nodes z < floor, its surface the plane z = floor - 1/2; because
    z is periodic the floor is also a ceiling, with the surface z = nz - 1/2. Each
    spacing x spacing cell holds one post on its centre axis: a cone frustum standing on
    the floor surface, radius r_base there, r_tip at the top, height `height`
    (r_base < spacing/2 - 1, so no link reaches a post across a cell edge). nx and ny must
    be multiples of spacing. Returns (mask uint8 [N], link_q (3,3,3,N)) with exact cut
    fractions as in sphere_obstacle.
    """
    if nx % spacing or ny % spacing:
        raise ValueError("nx and ny must be multiples of the post spacing")
    if not (0 < r_tip and 0 < r_base < 0.5 * spacing - 1):
        raise ValueError("post radii must be positive and below spacing/2 - 1")
    zf = floor - 0.5
    ztop = zf + height
    half = 0.5 * spacing
    slope = (r_tip - r_base) / height

    def phi_at(rx, ry, zw):
        # zw: height with the floor slab at [-1/2, zf] (a link across the top of the box
        # starts at zw = -1); rx, ry from the post axis; posts stand on the slab
        slab = np.maximum(zw - zf, -0.5 - zw)
        post = np.maximum(np.sqrt(rx * rx + ry * ry) - (r_base + slope * (zw - zf)),
                          np.maximum(zw - ztop, -0.5 - zw))
        return np.minimum(slab, post)

    def along(px, py, pz, c):
        rx = np.mod(px, spacing) - half         # the link's own cell: posts never cross an edge
        ry = np.mod(py, spacing) - half
        zw = np.where(pz + 0.5 * c[2] >= nz - 0.5, pz - nz, pz)   # the link crosses z = nz - 1/2
        return lambda t: phi_at(rx + t * c[0], ry + t * c[1], zw + t * c[2])

    x, y, z = _grid(nx, ny, nz)
    solid = phi_at(np.mod(x, spacing) - half, np.mod(y, spacing) - half, z) <= 0
    return solid.astype(np.uint8), _link_fractions(along, solid, (nx, ny, nz))


def channel_column(nx: int, H: int, wall: int, rho_liquid: float, rho_vapour: float, width: float,
                   x0: float, x1: float):
    """D2Q9 channel along x between solid rows: `wall` solid rows at the bottom and at the
    top, H fluid rows between them (ny = H + 2 wall), periodic in x. A liquid column fills
    x0 <= x < x1 across the whole channel, with tanh faces of width `width`; vapour
    elsewhere. Returns (mask uint8 [N], rho [N]); solid nodes carry rho_vapour."""
    ny = H + 2 * wall
    x, y, _ = _grid(nx, ny, 1)
    d = np.minimum(x - x0, x1 - x)
    rho = tanh_profile(d, rho_liquid, rho_vapour, width)
    solid = (y < wall) | (y >= ny - wall)
    return solid.astype(np.uint8), np.where(solid, rho_vapour, rho)


def random_state(N: int, D: int, rho_lo: float, rho_hi: float, umax: float, seed: int):
    """Random density in [rho_lo, rho_hi) and velocity components in [-umax, umax)."""
    u01 = (splitmix64(seed, N) >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)
    rho = rho_lo + (rho_hi - rho_lo) * u01
    u = np.stack([uniform_pm(seed + 7919 * (a + 1), N, umax) for a in range(D)])
    return rho, u


@dataclass(frozen=True)
class SweepCase:
    """One flat-interface case of the batched temperature sweep (D2Q9, ny x L periodic)."""
    index: int
    T_reduced: float
    nx: int          # length across the interface (x)
    ny: int          # width (y)
    fp64: bool


def temperature_sweep(ncases: int = 64, t_lo: float = 0.55, t_hi: float = 0.99,
                      l_lo: int = 128, l_hi: int = 2048, width: int = 4,
                      fp64_from: float = 0.95) -> list[SweepCase]:
    """Uniformly spaced reduced temperatures; lengths log-spaced and increasing with T."""
    cases = []
    for k in range(ncases):
        s = k / (ncases - 1) if ncases > 1 else 0.0
        tr = t_lo + (t_hi - t_lo) * s
        length = int(round(l_lo * (l_hi / l_lo) ** s))
        cases.append(SweepCase(k, tr, length, width, tr >= fp64_from))
    return cases


def impact_drop_velocity(rho: np.ndarray, rho_liquid: float, rho_vapour: float, D: int,
                         speed: float, axis: int) -> np.ndarray:
    """Velocity `speed` along `axis` weighted by the liquid fraction (drop-impact start)."""
    u = np.zeros((D, rho.size))
    u[axis] = speed * liquid_fraction(rho, rho_liquid, rho_vapour)
    return u


def log_spaced_int(lo: int, hi: int, count: int) -> list[int]:
    return [int(round(lo * (hi / lo) ** (k / (count - 1)))) for k in range(count)]


def equimolar_offset(profile: np.ndarray, rho_liquid: float, rho_vapour: float) -> float:
    """Position (in nodes from index 0) of the equimolar surface of a monotone
    vapour->liquid profile: the excess mass left of it equals the deficit right of it."""
    excess = float(np.sum(profile - rho_vapour))
    return len(profile) - excess / (rho_liquid - rho_vapour)


def radial_from_profile(nx: int, ny: int, nz: int, radius: float, profile: np.ndarray,
                        centre=None, noise: float = 0.0, seed: int = 0) -> np.ndarray:
    """Drop whose radial density follows a given 1D vapour->liquid profile.

    `profile` samples the density at unit spacing across one flat interface,
    vapour at index 0 and liquid at the end; its equimolar surface is placed at
    distance `radius` from the centre, and the ends are held constant beyond the
    sampled range.
    """
    profile = np.asarray(profile, dtype=np.float64)
    rv, rl = float(profile[0]), float(profile[-1])
    xe = equimolar_offset(profile, rl, rv)
    d_grid = np.arange(len(profile)) - xe + 0.5
    x, y, z = _grid(nx, ny, nz)
    if centre is None:
        centre = ((nx - 1) / 2.0, (ny - 1) / 2.0, (nz - 1) / 2.0)
    cx, cy, cz = centre
    r = np.sqrt((x - cx) ** 2 + (y - cy) ** 2 + ((z - cz) ** 2 if nz > 1 else 0.0))
    rho = np.interp(radius - r, d_grid, profile, left=rv, right=rl)
    return add_noise(rho, seed, noise)


__all__ = [
    "splitmix64", "uniform_pm", "tanh_profile", "add_noise", "flat_slab", "drop", "zero_velocity",
    "liquid_fraction", "pillar_mask", "random_mask", "random_state", "SweepCase", "temperature_sweep",
    "impact_drop_velocity", "log_spaced_int", "equimolar_offset", "radial_from_profile",
]
