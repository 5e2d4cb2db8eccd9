"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module holds no part of the method's arithmetic: it only produces initial
states (random numbers from a counter-based generator and closed-form initial
data) and moves interior values in and out of ghosted patch arrays.

Counter-based generator: SplitMix64 (Steele, Lea & Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014), keyed by
(seed, level, field, global i, j, k) so that a value does not depend on how a
level is cut into patches.

Patch array layout (the same convention on both sides of every comparison):
``(nf, nz+6, ny+6, nx+6)`` float64, x fastest, ghost width 3.
"""
from __future__ import annotations

import numpy as np

G = 3
_M64 = np.uint64(0xFFFFFFFFFFFFFFFF)


def _splitmix(x: np.ndarray) -> np.ndarray:
    with np.errstate(over="ignore"):
        z = x + np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def uniform(seed: int, level: int, field: int, gi, gj, gk) -> np.ndarray:
    """Uniform numbers in [-1, 1) keyed by the global point index (broadcasting)."""
    gi = np.asarray(gi, dtype=np.int64).astype(np.uint64)
    gj = np.asarray(gj, dtype=np.int64).astype(np.uint64)
    gk = np.asarray(gk, dtype=np.int64).astype(np.uint64)
    h = _splitmix(np.uint64(seed) & _M64)
    h = _splitmix(h ^ np.uint64(level))
    h = _splitmix(h ^ np.uint64(field))
    h = _splitmix(h ^ gi)
    h = _splitmix(h ^ gj)
    h = _splitmix(h ^ gk)
    u = (h >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)
    return 2.0 * u - 1.0


def embed(interior: np.ndarray) -> np.ndarray:
    """(nf, nz, ny, nx) interior values -> ghosted patch array (ghosts zero)."""
    nf, nz, ny, nx = interior.shape
    out = np.zeros((nf, nz + 2 * G, ny + 2 * G, nx + 2 * G))
    out[:, G:G + nz, G:G + ny, G:G + nx] = interior
    return out


def interior(patch: np.ndarray) -> np.ndarray:
    return patch[:, G:-G, G:-G, G:-G]


def grid(lo, n, dx):
    """Vertex-centred coordinates x_i = xlo + i dx of an interior box of size n
    starting at global index lo; returns broadcastable (z, y, x) arrays."""
    x = (lo[0] + np.arange(n[0])) * dx
    y = (lo[1] + np.arange(n[1])) * dx
    z = (lo[2] + np.arange(n[2])) * dx
    return z[:, None, None], y[None, :, None], x[None, None, :]


# ---------------------------------------------------------------- wave data

def wave_gaussian(n, xlo, dx, amp=1.0, width=0.2, centre=(0.0, 0.0, 0.0), lo=(0, 0, 0),
                  period=None):
    """phi = amp exp(-|x - c|^2 / width^2), Pi = 0 on a periodic box; the
    distance uses the minimum image when ``period`` (domain length per axis)
    is given.  Returns (2, nz, ny, nx)."""
    z, y, x = grid(lo, n, dx)
    x = x + xlo[0]
    y = y + xlo[1]
    z = z + xlo[2]
    d = [x - centre[0], y - centre[1], z - centre[2]]
    if period is not None:
        d = [di - period[i] * np.round(di / period[i]) for i, di in enumerate(d)]
    r2 = d[0] ** 2 + d[1] ** 2 + d[2] ** 2
    phi = amp * np.exp(-r2 / width ** 2)
    out = np.zeros((2,) + tuple(reversed(n)))
    out[0] = np.broadcast_to(phi, out[0].shape)
    return out


def wave_centre(seed: int):
    """Pulse centre drawn uniformly in [-0.3, 0.3]^3 from the generator."""
    return tuple(0.3 * float(uniform(seed, 99, 99, c, 0, 0)) for c in range(3))


# ----------------------------------------------------------------- MHD data

def mhd_ot_like(n, seed=0, p0=0.6, gamma=5.0 / 3.0, lo=(0, 0, 0), N=None):
    """Smooth periodic state on [0,1)^3 (conserved fields rho, S, E, B):
    rho = 1 + 1e-3 xi, p = p0,
    v = 0.5 (sin 2pi z - sin 2pi y, sin 2pi x - sin 2pi z, sin 2pi y - sin 2pi x),
    B = 0.3 (sin 4pi z - sin 2pi y, sin 4pi x - sin 2pi z, sin 4pi y - sin 2pi x)."""
    N = n if N is None else N
    dx = 1.0 / N[0]
    z, y, x = grid(lo, n, dx)
    s2 = lambda a: np.sin(2 * np.pi * a)
    s4 = lambda a: np.sin(4 * np.pi * a)
    shape = tuple(reversed(n))
    gk, gj, gi = np.meshgrid(lo[2] + np.arange(n[2]), lo[1] + np.arange(n[1]),
                             lo[0] + np.arange(n[0]), indexing="ij")
    rho = 1.0 + 1e-3 * uniform(seed, 0, 0, gi, gj, gk)
    v = [np.broadcast_to(0.5 * (s2(z) - s2(y)), shape),
         np.broadcast_to(0.5 * (s2(x) - s2(z)), shape),
         np.broadcast_to(0.5 * (s2(y) - s2(x)), shape)]
    B = [np.broadcast_to(0.3 * (s4(z) - s2(y)), shape),
         np.broadcast_to(0.3 * (s4(x) - s2(z)), shape),
         np.broadcast_to(0.3 * (s4(y) - s2(x)), shape)]
    v2 = v[0] ** 2 + v[1] ** 2 + v[2] ** 2
    B2 = B[0] ** 2 + B[1] ** 2 + B[2] ** 2
    E = 0.5 * rho * v2 + p0 / (gamma - 1.0) + 0.5 * B2
    out = np.zeros((8,) + shape)
    out[0] = rho
    for i in range(3):
        out[1 + i] = rho * v[i]
        out[5 + i] = B[i]
    out[4] = E
    return out


def mhd_primitive_to_conserved(rho, v, p, B, gamma):
    v2 = sum(vi * vi for vi in v)
    B2 = sum(b * b for b in B)
    out = np.zeros((8,) + np.shape(rho))
    out[0] = rho
    for i in range(3):
        out[1 + i] = rho * v[i]
        out[5 + i] = B[i]
    out[4] = 0.5 * rho * v2 + p / (gamma - 1.0) + 0.5 * B2
    return out


# ---------------------------------------------------------------- CCZ4 data

CCZ4_FLAT = np.array([1.0,                              # chi
                      1.0, 0.0, 0.0, 1.0, 0.0, 1.0,     # gt_ij
                      0.0,                              # trKhat
                      0.0, 0.0, 0.0, 0.0, 0.0, 0.0,     # At_ij
                      0.0, 0.0, 0.0,                    # Ghat^i
                      0.0,                              # Theta
                      1.0,                              # alpha
                      0.0, 0.0, 0.0,                    # beta^i
                      0.0, 0.0, 0.0])                   # B^i


def ccz4_minkowski_noise(n, amp=1e-10, seed=0, level=0, lo=(0, 0, 0)):
    """Minkowski (chi = alpha = 1, gt = delta, rest 0) plus amp * U[-1,1) noise
    on all 25 fields, keyed by global index."""
    shape = tuple(reversed(n))
    gk, gj, gi = np.meshgrid(lo[2] + np.arange(n[2]), lo[1] + np.arange(n[1]),
                             lo[0] + np.arange(n[0]), indexing="ij")
    out = np.empty((25,) + shape)
    for f in range(25):
        out[f] = CCZ4_FLAT[f] + amp * uniform(seed, level, f, gi, gj, gk)
    return out


def ccz4_lapse_pulse(n, xlo, dx, amp=0.1, width=0.2, centre=(0.0, 0.0, 0.0), lo=(0, 0, 0)):
    """Flat data with alpha = 1 + amp exp(-|x-c|^2/width^2) (pure gauge)."""
    z, y, x = grid(lo, n, dx)
    r2 = (x + xlo[0] - centre[0]) ** 2 + (y + xlo[1] - centre[1]) ** 2 + (z + xlo[2] - centre[2]) ** 2
    shape = tuple(reversed(n))
    out = np.empty((25,) + shape)
    for f in range(25):
        out[f] = CCZ4_FLAT[f]
    out[18] = 1.0 + amp * np.broadcast_to(np.exp(-r2 / width ** 2), shape)
    return out


# ------------------------------------------------------------ hierarchies

def composition(total: int, parts: int, lo: int, hi: int, rng) -> list[int]:
    """Random composition of `total` into `parts` integers in [lo, hi]."""
    assert parts * lo <= total <= parts * hi
    out = [total // parts] * parts
    for i in range(total % parts):
        out[i] += 1
    for _ in range(8 * parts):
        i, j = rng.integers(0, parts, 2)
        d = int(rng.integers(1, 9))
        if i != j and out[i] - d >= lo and out[j] + d <= hi:
            out[i] -= d
            out[j] += d
    return out


def tiled_boxes(start, sizes_per_axis):
    """Boxes tiling the region that starts at `start` with the given segment
    lengths per axis (x fastest)."""
    edges = []
    for d in range(3):
        e = [start[d]]
        for s in sizes_per_axis[d]:
            e.append(e[-1] + s)
        edges.append(e)
    boxes = []
    for k in range(len(sizes_per_axis[2])):
        for j in range(len(sizes_per_axis[1])):
            for i in range(len(sizes_per_axis[0])):
                lo = (edges[0][i], edges[1][j], edges[2][k])
                hi = (edges[0][i + 1] - 1, edges[1][j + 1] - 1, edges[2][k + 1] - 1)
                boxes.append((lo, hi))
    return boxes


def amr_three_levels(seed: int = 0):
    """Three-level hierarchy on [-1, 1)^3: level 0 = 128^3 tiled 4x4x4; level 1
    (ratio 2) = 128^3 fine points centred, tiled 4x4x4; level 2 (ratio 3) =
    192 x 132 x 96 fine points centred, tiled 6x4x3.  Segment lengths per
    axis are seeded random compositions with parts in [16, 48]; 200 patches."""
    rng = np.random.default_rng(seed)
    l0 = tiled_boxes((0, 0, 0), [composition(128, 4, 16, 48, rng) for _ in range(3)])
    l1 = tiled_boxes((64, 64, 64), [composition(128, 4, 16, 48, rng) for _ in range(3)])
    ext2 = (192, 132, 96)
    start2 = tuple((768 - e) // 2 for e in ext2)
    l2 = tiled_boxes(start2, [composition(ext2[0], 6, 16, 48, rng), composition(ext2[1], 4, 16, 48, rng),
                              composition(ext2[2], 3, 16, 48, rng)])
    return [(1, l0), (2, l1), (3, l2)], (128, 128, 128), 2.0 / 128


def wave_channel_pulse(x, t, L, width=0.173):
    """Exact scalar field of the FMR wave test (Sec. IV.A): a Gaussian of
    width `width` released at rest at x = 0 splits into halves moving left
    and right, on a periodic line of length L (nearest images summed)."""
    x = np.asarray(x, dtype=np.float64)
    g = lambda s: np.exp(-(s ** 2) / width ** 2)
    return sum(0.5 * (g(x - t + m * L) + g(x + t + m * L)) for m in (-1, 0, 1))


def mhd_cp_alfven(n, dx, lo=(0, 0, 0), L=2.0, gamma=5.0 / 3.0):
    """Circularly polarised Alfven wave of the MHD tests (Sec. IV.B.1) on a
    square periodic box of side L in x, y with alpha = pi/4: rho = 1, p = 0.1,
    B_par = 1, B_perp = v_perp = 0.1 sin(phase), B_z = v_z = 0.1 cos(phase),
    phase = 2 pi x_par / (L cos alpha) (one wavelength along k across the box),
    B_perp = B_y cos alpha - B_x sin alpha.  Points at x = (lo + i) dx."""
    ca = sa = np.sqrt(0.5)
    x = (lo[0] + np.arange(n[0])) * dx
    y = (lo[1] + np.arange(n[1])) * dx
    X, Y = np.meshgrid(x, y)
    ph = 2.0 * np.pi * (X * ca + Y * sa) / (L * ca)
    bp, bz = 0.1 * np.sin(ph), 0.1 * np.cos(ph)
    B = [ca - bp * sa, sa + bp * ca, bz]
    v = [-bp * sa, bp * ca, bz]
    shape = (n[2], n[1], n[0])
    bc = lambda a: np.broadcast_to(np.asarray(a, dtype=np.float64), shape)
    return mhd_primitive_to_conserved(bc(1.0), [bc(c) for c in v], bc(0.1), [bc(c) for c in B], gamma)


def mhd_brio_wu(n, dx, lo=(0, 0, 0), jumps=(0.5, 2.5), gamma=2.0):
    """Brio-Wu magnetic shock tube (Sec. IV.B.3) on a periodic line: the
    left state (rho 1, p 1, B_y 1) for x <= jumps[0] and x > jumps[1], the
    right state (rho 0.125, p 0.1, B_y -1) between; B_x = 0.75, v = B_z = 0."""
    x = (lo[0] + np.arange(n[0])) * dx
    left = (x <= jumps[0]) | (x > jumps[1])
    shape = (n[2], n[1], n[0])
    bc = lambda a: np.broadcast_to(np.asarray(a, dtype=np.float64), shape)
    rho = bc(np.where(left, 1.0, 0.125))
    p = bc(np.where(left, 1.0, 0.1))
    By = bc(np.where(left, 1.0, -1.0))
    zero = bc(0.0)
    return mhd_primitive_to_conserved(rho, [zero, zero, zero], p, [bc(0.75), By, zero], gamma)
