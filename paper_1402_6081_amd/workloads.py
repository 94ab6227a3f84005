"""Seeded synthetic inputs: block layouts and source fields.

This module holds input generation only (numpy PCG64 streams); it contains none of
the solver's arithmetic and is shared by the tests, the benchmark and the CPU checks.

Conventions used throughout the package:
  * a layout is an int32 array [N_B, 3] of block coordinates (bx, by, bz);
  * a field on a layout is an array [N_B, n, n, n] indexed [block, z, y, x] (x fastest);
    the grid point of entry (b, z, y, x) is (bx*n + x, by*n + y, bz*n + z).

Workload families (shapes after the paper's experiments, Sec. 4, and the vortex-ring
application of Sec. 5): cubes, spheres and thin spherical shells of blocks,
face-connected random layouts grown by an Eden process, Gaussian-bump sources, a thin
vortex-ring-shaped source, and random manufactured solutions (Sec. 4.1).
"""
import numpy as np

__all__ = [
    "cube_layout", "sphere_layout", "shell_layout", "eden_layout", "dilate_layout", "split_sets", "points_of",
    "gaussian_source", "zero_mean_gaussians", "vortex_ring_source", "random_manufactured",
    "boundary_mask", "manufactured_pair", "config_small", "config_medium", "config_large", "config_split",
    "config_scheme",
]


def cube_layout(nb):
    """All blocks of an nb^3 cube, lexicographic (x fastest)."""
    z, y, x = np.meshgrid(np.arange(nb), np.arange(nb), np.arange(nb), indexing="ij")
    return np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1).astype(np.int32)


def sphere_layout(nb):
    """Blocks of an nb^3 box whose centres lie inside the inscribed sphere."""
    c = cube_layout(nb).astype(np.float64) + 0.5
    r = np.linalg.norm(c - nb / 2.0, axis=1)
    return cube_layout(nb)[r <= nb / 2.0]


def shell_layout(nb, thickness=0.1):
    """Blocks whose centres lie in a spherical shell of the given thickness (fraction
    of the diameter), as in the paper's shell geometry (Sec. 4.2)."""
    c = cube_layout(nb).astype(np.float64) + 0.5
    r = np.linalg.norm(c - nb / 2.0, axis=1)
    R = nb / 2.0
    keep = (r <= R) & (r >= R - thickness * nb - 0.5)
    return cube_layout(nb)[keep]


def eden_layout(nblocks, rng, max_extent=None):
    """Face-connected random set of `nblocks` blocks grown from the origin by an Eden
    process (each step activates a uniformly chosen face neighbour of the set)."""
    cur = {(0, 0, 0)}
    frontier = []

    def push(b):
        for d in ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)):
            nb = (b[0] + d[0], b[1] + d[1], b[2] + d[2])
            if nb in cur:
                continue
            if max_extent is not None and max(abs(v) for v in nb) >= max_extent:
                continue
            frontier.append(nb)

    push((0, 0, 0))
    while len(cur) < nblocks and frontier:
        i = int(rng.integers(len(frontier)))
        b = frontier[i]
        frontier[i] = frontier[-1]
        frontier.pop()
        if b in cur:
            continue
        cur.add(b)
        push(b)
    arr = np.array(sorted(cur, key=lambda t: (t[2], t[1], t[0])), dtype=np.int64)
    arr -= arr.min(axis=0)
    return arr.astype(np.int32)


def eden_box_layout(edge, fill, rng):
    """Face-connected Eden cluster of round(fill * edge^3) blocks grown from the centre of
    an edge^3 box and confined to it (bounding-box edge <= `edge`)."""
    target = max(1, int(round(fill * edge ** 3)))
    c = (edge // 2,) * 3
    cur = {c}
    frontier = []

    def push(b):
        for d in ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)):
            nb = (b[0] + d[0], b[1] + d[1], b[2] + d[2])
            if nb not in cur and all(0 <= v < edge for v in nb):
                frontier.append(nb)

    push(c)
    while len(cur) < target and frontier:
        i = int(rng.integers(len(frontier)))
        b = frontier[i]
        frontier[i] = frontier[-1]
        frontier.pop()
        if b in cur:
            continue
        cur.add(b)
        push(b)
    arr = np.array(sorted(cur, key=lambda t: (t[2], t[1], t[0])), dtype=np.int64)
    arr -= arr.min(axis=0)
    return arr.astype(np.int32)


def serving_mix(count, rng, n=16):
    """Request layouts of the serving workload: bounding-box edge U{2..16} blocks, Eden
    fill U[0.3, 1.0], each with max(1, N_B / 8) zero-net Gaussians (sigma U[2, 6])."""
    out = []
    for _ in range(count):
        edge = int(rng.integers(2, 17))
        fill = float(rng.uniform(0.3, 1.0))
        b = eden_box_layout(edge, fill, rng)
        f, _ = zero_mean_gaussians(b, n, rng, max(1, b.shape[0] // 8))
        out.append((b, f))
    return out


def dilate_layout(blocks, r=1):
    """Blocks within Chebyshev distance r of a block of the layout (the layout plus an
    r-block halo), sorted z, y, x."""
    s = {tuple(b) for b in np.asarray(blocks).tolist()}
    rng_ = range(-r, r + 1)
    out = {(x + dx, y + dy, z + dz) for (x, y, z) in s for dx in rng_ for dy in rng_ for dz in rng_}
    return np.array(sorted(out, key=lambda t: (t[2], t[1], t[0])), dtype=np.int32)


def split_sets(kind, rng):
    """(source blocks, evaluation blocks) of the three shapes separate sets take:
    "dilated"  sources on a small Eden cluster, evaluation on it plus a one-block halo;
    "subset"   evaluation on 7 of the 30 blocks of a source cluster;
    "disjoint" a source cluster and a shifted evaluation cluster with the overlap removed."""
    if kind == "dilated":
        src = eden_layout(14, rng)
        return src, dilate_layout(src, 1)
    if kind == "subset":
        src = eden_layout(30, rng)
        pick = rng.choice(len(src), size=7, replace=False)
        return src, src[np.sort(pick)]
    if kind == "disjoint":
        src = eden_layout(12, rng)
        ev = eden_layout(10, rng) + np.array([6, 1, -2], dtype=np.int32)
        s = {tuple(b) for b in src.tolist()}
        return src, np.asarray([b for b in ev.tolist() if tuple(b) not in s], dtype=np.int32)
    raise ValueError(kind)


def points_of(blocks, n):
    """Grid coordinates [N_B, n, n, n, 3] (x, y, z) of every point of every block."""
    b = np.asarray(blocks, dtype=np.int64)
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    local = np.stack([x, y, z], axis=-1)
    return b[:, None, None, None, :] * n + local[None]


def _axis_factors(blocks, n, centres, sigmas):
    """Per-block 1D factors of exp(-|x - c|^2 / (2 sigma^2)) = ex(x) ey(y) ez(z):
    E[d] has shape [N_B, G, n] (axis d = x, y, z)."""
    b = np.asarray(blocks, dtype=np.int64)
    c = np.atleast_2d(np.asarray(centres, dtype=np.float64))
    s = np.atleast_1d(np.asarray(sigmas, dtype=np.float64))
    out = []
    for d in range(3):
        coord = (b[:, d, None] * n + np.arange(n)[None, :]).astype(np.float64)  # [N_B, n]
        out.append(np.exp(-(coord[:, None, :] - c[None, :, d, None]) ** 2 / (2.0 * s[None, :, None] ** 2)))
    return out


def _sum_separable(E, amps):
    """f[b, z, y, x] = sum_g amps[g] ez[b, g, z] ey[b, g, y] ex[b, g, x]."""
    ex, ey, ez = E
    nb, g, n = ex.shape
    out = np.empty((nb, n, n, n))
    a = np.asarray(amps)[None, :, None]
    for b0 in range(0, nb, 128):  # chunks of blocks bound the [chunk, G, n, n] temporary
        b1 = min(nb, b0 + 128)
        zy = (ez[b0:b1] * a)[:, :, :, None] * ey[b0:b1, :, None, :]          # [c, G, z, y]
        zy = zy.reshape(b1 - b0, g, n * n).transpose(0, 2, 1)                # [c, zy, G]
        out[b0:b1] = np.matmul(zy, ex[b0:b1]).reshape(b1 - b0, n, n, n)
    return out


def gaussian_source(blocks, n, centres, sigmas, amps):
    """sum_g amps[g] exp(-|x - c_g|^2 / (2 sigma_g^2)) sampled on the layout's points."""
    return _sum_separable(_axis_factors(blocks, n, centres, sigmas), amps)


def zero_mean_gaussians(blocks, n, rng, count, sigma_lo=2.0, sigma_hi=6.0):
    """`count` Gaussians with centres uniform over the layout's bounding box, sigma
    ~ U[sigma_lo, sigma_hi], amplitudes N(0,1), then scaled so the net source is 0:
    the least-squares multiple of each bump's own discrete mass is removed, i.e.
    amps <- amps - m (m . amps) / (m . m) with m_g the sampled mass of bump g."""
    b = np.asarray(blocks)
    lo = b.min(axis=0) * n
    hi = (b.max(axis=0) + 1) * n
    centres = lo + rng.random((count, 3)) * (hi - lo)
    sigmas = rng.uniform(sigma_lo, sigma_hi, count)
    amps = rng.standard_normal(count)
    E = _axis_factors(blocks, n, centres, sigmas)
    mass = np.einsum("bg,bg,bg->g", E[0].sum(axis=2), E[1].sum(axis=2), E[2].sum(axis=2))
    amps = amps - mass * (mass @ amps) / (mass @ mass)
    return _sum_separable(E, amps), dict(centres=centres, sigmas=sigmas, amps=amps)


def _random_rotation(rng):
    q = rng.standard_normal(4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])


def vortex_ring_source(blocks, n, rng, radius=80.0, core=4.0, component=0):
    """Thin vortex-ring-shaped source: one Cartesian component of the vorticity of a
    ring of the given radius with a Gaussian core, centred in the layout's bounding
    box, normal tilted by a seeded random rotation.  The component of the unit
    tangent gives a field with (near) zero net source."""
    b = np.asarray(blocks)
    centre = (b.min(axis=0) * n + (b.max(axis=0) + 1) * n) / 2.0
    Rm = _random_rotation(rng)
    P = points_of(blocks, n).astype(np.float64) - centre
    Q = P @ Rm  # coordinates in the ring frame (ring in the local x-y plane)
    rho = np.sqrt(Q[..., 0] ** 2 + Q[..., 1] ** 2)
    d2 = (rho - radius) ** 2 + Q[..., 2] ** 2
    amp = np.exp(-d2 / (2.0 * core * core))
    safe = np.where(rho > 0, rho, 1.0)
    tang_local = np.stack([-Q[..., 1] / safe, Q[..., 0] / safe, np.zeros_like(rho)], axis=-1)
    tang = tang_local @ Rm.T
    return amp * tang[..., component]


def boundary_mask(blocks, n):
    """True at active points with at least one of the 6 lattice neighbours outside
    the active grid (the paper's boundary points, Sec. 4.1)."""
    b = np.asarray(blocks, dtype=np.int64)
    lo = b.min(axis=0)
    ext = b.max(axis=0) - lo + 1
    occ = np.zeros((ext[2] * n + 2, ext[1] * n + 2, ext[0] * n + 2), dtype=bool)
    for (bx, by, bz) in (b - lo).tolist():
        occ[1 + bz * n:1 + (bz + 1) * n, 1 + by * n:1 + (by + 1) * n, 1 + bx * n:1 + (bx + 1) * n] = True
    inner = (occ[2:, 1:-1, 1:-1] & occ[:-2, 1:-1, 1:-1] & occ[1:-1, 2:, 1:-1] & occ[1:-1, :-2, 1:-1]
             & occ[1:-1, 1:-1, 2:] & occ[1:-1, 1:-1, :-2])
    mask = np.zeros((b.shape[0], n, n, n), dtype=bool)
    for i, (bx, by, bz) in enumerate((b - lo).tolist()):
        mask[i] = ~inner[bz * n:(bz + 1) * n, by * n:(by + 1) * n, bx * n:(bx + 1) * n]
    return mask


def random_manufactured(blocks, n, rng):
    """u_rand ~ U[-1, 1] on the active grid, 0 on its boundary points (Sec. 4.1)."""
    u = rng.uniform(-1.0, 1.0, (len(blocks), n, n, n))
    u[boundary_mask(blocks, n)] = 0.0
    return u


def manufactured_pair(blocks, n, rng):
    """(u_rand, f = L u_rand) of Sec. 4.1: u_rand ~ U[-1, 1] on the active grid, 0 on its
    boundary points, and f its 7-point Laplacian [L u](x) = sum_{+-e_i} u(x +- e_i) - 6 u(x),
    which vanishes off the active grid, so G * f = u_rand exactly."""
    b = np.asarray(blocks, dtype=np.int64)
    lo = b.min(axis=0)
    ext = b.max(axis=0) - lo + 1
    u = random_manufactured(blocks, n, rng)
    D = np.zeros((ext[2] * n + 2, ext[1] * n + 2, ext[0] * n + 2))
    for i, (bx, by, bz) in enumerate((b - lo).tolist()):
        D[1 + bz * n:1 + (bz + 1) * n, 1 + by * n:1 + (by + 1) * n, 1 + bx * n:1 + (bx + 1) * n] = u[i]
    Lu = (D[2:, 1:-1, 1:-1] + D[:-2, 1:-1, 1:-1] + D[1:-1, 2:, 1:-1] + D[1:-1, :-2, 1:-1]
          + D[1:-1, 1:-1, 2:] + D[1:-1, 1:-1, :-2] - 6.0 * D[1:-1, 1:-1, 1:-1])
    f = np.empty_like(u)
    for i, (bx, by, bz) in enumerate((b - lo).tolist()):
        f[i] = Lu[bz * n:(bz + 1) * n, by * n:(by + 1) * n, bx * n:(bx + 1) * n]
    return u, f


# ----------------------------------------------------------------------------- named workloads

def config_small(seed=0):
    """32^3 cube as 4^3 blocks of 8^3, p = 6, 2 levels, FP64; 4 Gaussians (sigma = 3,
    centres uniform over the cube, amplitudes U[-1, 1])."""
    rng = np.random.default_rng(seed)
    blocks = cube_layout(4)
    n = 8
    centres = rng.random((4, 3)) * 32.0
    amps = rng.uniform(-1.0, 1.0, 4)
    f = gaussian_source(blocks, n, centres, np.full(4, 3.0), amps)
    return dict(blocks=blocks, n=n, p=6, levels=2, f=f, name="cube32_n8_p6_L2")


def config_medium(seed=1):
    """128^3 cube as 8^3 blocks of 16^3, p = 8, 4 levels; 32 Gaussians with sigma in
    U[2, 6], amplitudes N(0, 1) scaled to zero net source."""
    rng = np.random.default_rng(seed)
    blocks = cube_layout(8)
    n = 16
    f, _ = zero_mean_gaussians(blocks, n, rng, 32)
    return dict(blocks=blocks, n=n, p=8, levels=4, f=f, name="cube128_n16_p8_L4")


def config_large(seed=2):
    """256^3 cube as 16^3 blocks of 16^3, p = 8, full depth; thin vortex-ring source
    (R = 80, core sigma = 4, seeded tilt)."""
    rng = np.random.default_rng(seed)
    blocks = cube_layout(16)
    n = 16
    f = vortex_ring_source(blocks, n, rng)
    return dict(blocks=blocks, n=n, p=8, levels=0, f=f, name="cube256_n16_p8_vortexring")


def config_split(seed=2):
    """Separate source and evaluation blocks on the 256^3 vortex-ring workload: sources on
    the blocks of the 16^3-block cube where the ring's field exceeds 1e-16 of its peak
    (779 blocks, f restricted to them), evaluation on all 4096 blocks; n = 16, p = 8,
    full depth."""
    c = config_large(seed)
    amp = np.max(np.abs(c["f"]), axis=(1, 2, 3))
    keep = amp > 1e-16 * amp.max()
    return dict(blocks=c["blocks"][keep], f=c["f"][keep], eval_blocks=c["blocks"], n=c["n"], p=c["p"],
                levels=c["levels"], name="ring256_split_n16_p8_full")


def config_scheme(seed=6):
    """The paper's own scheme family on the 128^3 cube (8^3 blocks of 16^3): n_I = n + 1 = 17
    nodes per interval edge, n_max = 10, full depth; a random manufactured solution
    (Sec. 4.1), so the exact u is known."""
    rng = np.random.default_rng(seed)
    blocks = cube_layout(8)
    u, f = manufactured_pair(blocks, 16, rng)
    return dict(blocks=blocks, n=16, p=17, levels=0, f=f, u_exact=u, name="cube128_n16_nI17_manufactured")
