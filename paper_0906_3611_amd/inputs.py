"""Seeded synthetic initial conditions for the two-species lattice.

This module draws random numbers and lays out initial density fields; it holds
none of the lattice Boltzmann arithmetic.  Both the GPU library's callers and
the CPU reference take their inputs from here, so the two always start from
bit-identical fields.

Random numbers come from the counter-based use of SplitMix64 (Steele, Lea and
Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014): the
k-th output (k = 1, 2, ...) of a generator seeded with ``seed`` is the
finalizer applied to ``seed + k * 0x9E3779B97F4A7C15`` (mod 2^64), and a
uniform double in [0, 1) is its top 53 bits times 2^-53.
"""
from __future__ import annotations

import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

# Counter offset of the disc draws, so they never overlap the per-site noise
# counters of any lattice that fits in memory.
DISC_COUNTER_BASE = 1 << 48


def splitmix64(seed: int, counters) -> np.ndarray:
    """Outputs number ``counters`` (1-based) of SplitMix64 seeded with ``seed``."""
    k = np.asarray(counters, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed % (1 << 64)) + k * _GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform01(seed: int, counters) -> np.ndarray:
    """Uniform doubles in [0, 1): (splitmix64 >> 11) * 2^-53, exact in FP64."""
    z = splitmix64(seed, counters)
    return (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def noise_fields(nx: int, ny: int, seed: int, mean_a: float, mean_b: float, amp: float):
    """Densities mean_s + amp (2U - 1), U i.i.d. per site and species.

    The draw for species s at (x, y) is output number (s*ny + y)*nx + x + 1 of
    the generator.  Returns (rho_a, rho_b), each (ny, nx) float64."""
    n = nx * ny
    out = []
    for s, mean in enumerate((mean_a, mean_b)):
        idx = np.arange(n, dtype=np.uint64) + np.uint64(s * n + 1)
        u = uniform01(seed, idx).reshape(ny, nx)
        out.append(mean + amp * (2.0 * u - 1.0))
    return out[0], out[1]


def noise_window(nx: int, ny: int, seed: int, mean_a: float, mean_b: float, amp: float,
                 x0: int, y0: int, w: int, h: int):
    """The (h, w) window of noise_fields(nx, ny, seed, ...) whose first site
    is (x0, y0): rows y0 .. y0+h-1 and columns x0 .. x0+w-1, both taken
    modulo the lattice.  The same draws, without generating the lattice."""
    xs = ((x0 + np.arange(w)) % nx).astype(np.uint64)
    ys = ((y0 + np.arange(h)) % ny).astype(np.uint64)
    out = []
    for s, mean in enumerate((mean_a, mean_b)):
        idx = (np.uint64(s) * np.uint64(ny) + ys[:, None]) * np.uint64(nx) + xs[None, :] + np.uint64(1)
        u = uniform01(seed, idx)
        out.append(mean + amp * (2.0 * u - 1.0))
    return out[0], out[1]


def disc_mask(nx: int, ny: int, seed: int, phi: float, rmin: float = 6.0, rmax: float = 12.0,
              max_discs: int = 10_000_000) -> np.ndarray:
    """Boolean (ny, nx) mask of the union of random discs covering >= phi.

    Disc k has centre (X, Y) = (nx U0, ny U1) and radius rmin + (rmax - rmin) U2,
    U_j = draw DISC_COUNTER_BASE + 3k + j + 1.  A site (x, y) is inside when its
    minimum-image periodic distance to the centre is <= the radius.  Discs are
    added until the covered fraction reaches phi."""
    if not (0.0 <= phi <= 1.0):
        raise ValueError("phi must lie in [0, 1]")
    mask = np.zeros((ny, nx), dtype=bool)
    target = phi * nx * ny
    covered = 0
    k = 0
    batch = 256
    while covered < target:
        if k >= max_discs:
            raise RuntimeError("disc placement did not reach the requested fraction")
        cnt = DISC_COUNTER_BASE + 3 * (k + np.arange(batch, dtype=np.int64))
        u0 = uniform01(seed, cnt + 1)
        u1 = uniform01(seed, cnt + 2)
        u2 = uniform01(seed, cnt + 3)
        for j in range(batch):
            cx, cy = nx * u0[j], ny * u1[j]
            r = rmin + (rmax - rmin) * u2[j]
            ri = int(np.ceil(r)) + 1
            xs = np.arange(int(np.floor(cx)) - ri, int(np.floor(cx)) + ri + 2)
            ys = np.arange(int(np.floor(cy)) - ri, int(np.floor(cy)) + ri + 2)
            dx = xs - cx
            dy = ys - cy
            # minimum image in each axis, then wrap the site index
            dx = dx - nx * np.round(dx / nx)
            dy = dy - ny * np.round(dy / ny)
            inside = (dy[:, None] ** 2 + dx[None, :] ** 2) <= r * r
            xi = np.mod(xs, nx)
            yi = np.mod(ys, ny)
            sub = mask[np.ix_(yi, xi)]
            newly = inside & ~sub
            if newly.any():
                # duplicate indices (tiny lattices) are harmless: OR is idempotent
                mask[np.ix_(yi, xi)] = sub | inside
                if len(xs) <= nx and len(ys) <= ny:
                    covered += int(newly.sum())
                else:
                    covered = int(mask.sum())
            k += 1
            if covered >= target:
                break
    return mask


def disc_fields(nx: int, ny: int, seed: int, phi: float, rmin: float = 6.0, rmax: float = 12.0,
                in_a: float = 1.2, in_b: float = 0.05, out_a: float = 0.05, out_b: float = 1.2):
    """Sharp two-phase emulsion: (in_a, in_b) inside the discs of disc_mask,
    (out_a, out_b) outside.  Returns (rho_a, rho_b), each (ny, nx) float64."""
    m = disc_mask(nx, ny, seed, phi, rmin, rmax)
    rho_a = np.where(m, in_a, out_a).astype(np.float64)
    rho_b = np.where(m, in_b, out_b).astype(np.float64)
    return rho_a, rho_b


def _uniform_stream(seed: int, base: int, n: int) -> np.ndarray:
    return uniform01(seed, np.uint64(base) + np.arange(1, n + 1, dtype=np.uint64))


ENSEMBLE_COUNTER_BASE = 1 << 52
TRACE_COUNTER_BASE = 1 << 53


def ensemble_specs(n: int = 256, seed: int = 4, lmin: int = 128, lmax: int = 1024,
                   ga_range=(-9.5, -8.5), phi_range=(0.5, 0.8)):
    """An ensemble of independent square lattices: side L = round(exp(U[ln lmin,
    ln lmax])), first-belt coupling G^a ~ U[ga_range] (both species), disc
    volume fraction phi ~ U[phi_range].  Returns a list of dicts
    (L, G_a, phi, seed) with a distinct disc seed per lattice."""
    u = _uniform_stream(seed, ENSEMBLE_COUNTER_BASE, 3 * n).reshape(n, 3)
    out = []
    for k in range(n):
        L = int(round(np.exp(np.log(lmin) + (np.log(lmax) - np.log(lmin)) * u[k, 0])))
        ga = ga_range[0] + (ga_range[1] - ga_range[0]) * u[k, 1]
        phi = phi_range[0] + (phi_range[1] - phi_range[0]) * u[k, 2]
        out.append({"L": L, "G_a": float(ga), "phi": float(phi), "seed": seed * 100003 + k})
    return out


def serving_trace(n: int, rate: float, seed: int = 5, side=(64, 2048), steps=(1000, 50000),
                  wall_speeds=(0.001, 0.005, 0.02)):
    """A finite arrival trace: Poisson arrivals of the given rate (jobs/s),
    half Couette jobs (wall speed drawn from wall_speeds) and half periodic,
    square sides and step counts log-uniform in the given ranges.  Returns a
    list of dicts (t, L, steps, boundary, u_wall, seed)."""
    u = _uniform_stream(seed, TRACE_COUNTER_BASE, 5 * n).reshape(n, 5)
    t = np.cumsum(-np.log1p(-u[:, 0]) / rate)
    out = []
    for k in range(n):
        L = int(round(np.exp(np.log(side[0]) + (np.log(side[1]) - np.log(side[0])) * u[k, 1])))
        st = int(round(np.exp(np.log(steps[0]) + (np.log(steps[1]) - np.log(steps[0])) * u[k, 2])))
        couette = u[k, 3] < 0.5
        uw = float(wall_speeds[min(int(u[k, 4] * len(wall_speeds)), len(wall_speeds) - 1)])
        out.append({"t": float(t[k]), "L": L, "steps": st,
                    "boundary": "couette" if couette else "periodic",
                    "u_wall": uw if couette else 0.0, "seed": seed * 1000003 + k})
    return out
