"""Seeded synthetic inputs of the benchmark workloads.

Pure data generation shared by the tests, the benchmark and both sides of a
parity check: obstacle layouts, particle placements, initial velocity fields
and domain-size mixes.  Nothing here evaluates the lattice-Boltzmann method
(no equilibria, no collision, no streaming); each side turns these inputs into
populations itself.

The paper's benchmark geometries exist only as figures, so these seeded
stand-ins have the shapes, sizes and structure of its workloads (disordered
disc packings, a block of closely spaced particles, a channel, periodic boxes).
"""
import numpy as np

BASE_SEED = 2006_12910


def rng(seed_offset=0):
    return np.random.default_rng(BASE_SEED + int(seed_offset))


def rsa_discs(nx, ny, rmin, rmax, solid_fraction, gap, rng_, x_margin=(0, 0), y_margin=(0, 0),
              periodic=False, max_tries=200000):
    """Random sequential addition of non-overlapping discs with radii uniform in
    [rmin, rmax] until the rasterised solid fraction (nodes with
    |x - c|^2 < r^2) reaches `solid_fraction`.  A candidate is rejected if its
    surface gap to an existing disc (or to a margin edge / the domain edge when
    not periodic) is below `gap`.  Returns (mask [ny][nx] uint8, discs [(x, y, r)])."""
    mask = np.zeros((ny, nx), np.uint8)
    cxs, cys, rs = np.empty(0), np.empty(0), np.empty(0)
    target = solid_fraction * nx * ny
    solid = 0
    x_lo, x_hi = x_margin[0], nx - x_margin[1]
    y_lo, y_hi = y_margin[0], ny - y_margin[1]
    tries = 0
    while solid < target and tries < max_tries:
        tries += 1
        r = rng_.uniform(rmin, rmax)
        if periodic:
            cx, cy = rng_.uniform(x_lo, x_hi), rng_.uniform(y_lo, y_hi)
        else:
            if x_hi - x_lo <= 2 * (r + gap) or y_hi - y_lo <= 2 * (r + gap):
                continue
            cx = rng_.uniform(x_lo + r + gap, x_hi - r - gap)
            cy = rng_.uniform(y_lo + r + gap, y_hi - r - gap)
        if rs.size:
            dx, dy = cx - cxs, cy - cys
            if periodic:
                dx -= nx * np.round(dx / nx)
                dy -= ny * np.round(dy / ny)
            if np.any(dx * dx + dy * dy < (r + rs + gap) ** 2):
                continue
        cxs, cys, rs = np.append(cxs, cx), np.append(cys, cy), np.append(rs, r)
        x0, x1 = int(np.floor(cx - r)) - 1, int(np.ceil(cx + r)) + 2
        y0, y1 = int(np.floor(cy - r)) - 1, int(np.ceil(cy + r)) + 2
        ys, xs = np.mgrid[y0:y1, x0:x1]
        inside = (xs - cx) ** 2 + (ys - cy) ** 2 < r * r
        xs, ys = xs[inside], ys[inside]
        if periodic:
            xs, ys = xs % nx, ys % ny
        else:
            keep = (xs >= 0) & (xs < nx) & (ys >= 0) & (ys < ny)
            xs, ys = xs[keep], ys[keep]
        solid += int((mask[ys, xs] == 0).sum())
        mask[ys, xs] = 1
    discs = list(zip(cxs.tolist(), cys.tolist(), rs.tolist()))
    return mask, discs


def porous_channel(nx=2048, ny=1024, seed=0, solid_fraction=0.35, inlet_margin=112,
                   outlet_margin=64):
    """Fractured porous medium: walls on y = 0 and ny-1, RSA discs r ~ U[6, 24]
    at the target solid fraction with gap >= 2, obstacle-free inlet/outlet
    margins; returns (mask, discs).  The wall rows are not part of the mask."""
    r = rng(100 + seed)
    mask, discs = rsa_discs(nx, ny, 6.0, 24.0, solid_fraction, 2.0, r,
                            x_margin=(inlet_margin, outlet_margin), y_margin=(1, 1))
    return mask, discs


def particle_block(rows=4, cols=4, radius=8.0, gap_x=8.5, gap_y=5.5, x0=12.5, y_centre=512.0):
    """A block of closely spaced discs (surface spacings gap_x horizontally and
    gap_y vertically), centres at half-integers offset by a quarter node so no
    node lies exactly on a surface; returns a list of (x, y)."""
    pitch_x, pitch_y = 2 * radius + gap_x, 2 * radius + gap_y
    out = []
    y0 = y_centre - 0.5 * (rows - 1) * pitch_y
    for i in range(rows):
        for j in range(cols):
            out.append((x0 + radius + j * pitch_x + 0.25, y0 + i * pitch_y + 0.25))
    return out


def shear_wave_field(nx, ny, amplitude, k, phase):
    """u_x = amplitude sin(2 pi k y / ny + phase), u_y = 0, rho = 1."""
    y = np.arange(ny, dtype=np.float64)
    ux = np.repeat((amplitude * np.sin(2 * np.pi * k * y / ny + phase))[:, None], nx, axis=1)
    return np.ones((ny, nx)), ux, np.zeros((ny, nx))


def log_uniform_sizes(count, smin, smax, seed=0):
    """Square domain sides log-uniform in [smin, smax], rounded to integers."""
    r = rng(300 + seed)
    return [int(round(smin * (smax / smin) ** r.uniform())) for _ in range(count)]


def stress_batch(count=200, seed=0, smin=64, smax=2048):
    """The uneven-domain ensemble: per domain its side, tau ~ U[0.55, 1.2],
    shear-wave number k in {1..4} and phase ~ U[0, 2 pi), and the seed of its
    RSA obstacle layout (discs r ~ U[3, 12], periodic, gap >= 1, 20% solid)."""
    sizes = log_uniform_sizes(count, smin, smax, seed)
    r = rng(400 + seed)
    out = []
    for i, n in enumerate(sizes):
        out.append(dict(n=n, tau=float(r.uniform(0.55, 1.2)), k=int(r.integers(1, 5)),
                        phase=float(r.uniform(0, 2 * np.pi)), obstacle_seed=1000 + 7 * i + seed))
    return out


def stress_obstacles(n, obstacle_seed, solid_fraction=0.20):
    mask, _ = rsa_discs(n, n, 3.0, 12.0, solid_fraction, 1.0, rng(obstacle_seed), periodic=True)
    return mask


def fluctuating_batch(count=64, seed=0, smin=128, smax=1024):
    """Ensemble of fluctuating-fluid realisations: sides log-uniform in
    [smin, smax], one disc of radius 5 at the centre (offset to (c + 0.5)),
    its own domain id per realisation."""
    sizes = log_uniform_sizes(count, smin, smax, 500 + seed)
    return [dict(n=n, domain_id=i + 1, disc=(n / 2 + 0.5, n / 2 + 0.5, 5.0))
            for i, n in enumerate(sizes)]


# The paper's three timing benchmarks (its Table of MLUPS), as seeded
# stand-ins: the lattices and parameters it states, with the geometry it shows
# only in figures replaced by the layouts below.

def replica_b1(seed=0, nx=1020, ny=1620, band=220, solid_fraction=0.30):
    """Multi-particle flow in a porous medium: lateral walls on x = 0 and
    nx-1 (not in the mask), periodic in y, RSA grains r ~ U[6, 24] (gap >= 2)
    to `solid_fraction` of the lattice outside a grain-free release band of
    `band` rows at the top, and 45 particles of radius 6.5 in three rows of 15
    in that band, surface spacings 8.5 horizontally and 5.5 vertically.
    Returns (mask, particle centres)."""
    r = rng(600 + seed)
    mask, _ = rsa_discs(nx, ny, 6.0, 24.0, solid_fraction, 2.0, r, x_margin=(1, 1),
                        y_margin=(0, band))
    radius, cols = 6.5, 15
    width = cols * (2 * radius + 8.5) - 8.5
    centres = particle_block(rows=3, cols=cols, radius=radius, gap_x=8.5, gap_y=5.5,
                             x0=0.5 * (nx - width), y_centre=ny - 0.5 * band)
    return mask, centres


def replica_b2(nx=3000, ny=41):
    """Brownian particle in a smooth channel: one disc of radius 7.5 at the
    channel centre (half-integer centre, so no node lies on its surface)."""
    return [(nx / 2 + 0.5, (ny - 1) / 2 + 0.5)]
