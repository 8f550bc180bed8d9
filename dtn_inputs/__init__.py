"""Seeded synthetic inputs for the local DtN workloads.

This module only *describes* inputs: domains, Dirichlet data, the list of
patches a caller asks Neumann data for, seeds, random interior points and
targets.  It holds none of the method's arithmetic (no nodes, walks, Green's
functions or quadratures); both the HIP library's callers and the oracle read
the same descriptions from here.

Domains and data follow the paper's workloads in kind: exact harmonic
Dirichlet data (a harmonic quadratic, or sums of q/|x - s| with sources
outside the domain), so that the exact Neumann data is known.

Patch description (one row per patch, arrays of length P):
  c [P,3]   patch centre on the boundary
  n [P,3]   outward unit normal of the domain at c
  t1 [P,3]  unit tangent; the second tangent is t2 = n x t1
  h [P]     hemisphere radius (also the radius of the patch S)
  n_theta, n_phi, n_rings, n_sectors [P]  node grid and panel layout
"""
import numpy as np

# ----------------------------------------------------------------- domains


def geometry_ball_quadratic(eps=1e-4, max_steps=1_000_000):
    """Unit ball, u = x^2 - y^2 + z (harmonic)."""
    quad = [0.0, 0.0, 0.0, 1.0, 1.0, -1.0, 0.0, 0.0, 0.0, 0.0]
    return {"kind": "ball", "ball_c": (0.0, 0.0, 0.0), "ball_r": 1.0,
            "data_kind": "quadratic", "quad": quad, "src": np.zeros((0, 4)),
            "holes": np.zeros((0, 6)), "eps": eps, "max_steps": max_steps}


def cube_sources(seed=2, n_src=8, centre=(0.5, 0.5, 0.5), r_in=1.5, r_out=3.0):
    """Point sources uniform in volume in a spherical shell around the cube
    centre, charges U(-1, 1).  Rows are (x, y, z, q)."""
    rng = np.random.default_rng(seed)
    u = rng.random(n_src)
    r = (r_in ** 3 + u * (r_out ** 3 - r_in ** 3)) ** (1.0 / 3.0)
    d = rng.standard_normal((n_src, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    q = rng.uniform(-1.0, 1.0, n_src)
    s = np.asarray(centre)[None, :] + r[:, None] * d
    return np.ascontiguousarray(np.column_stack([s, q]))


def geometry_cube_sources(seed=2, eps=1e-5, max_steps=1_000_000):
    """Unit cube [0,1]^3 with u = sum_k q_k / |x - s_k|, 8 exterior sources."""
    return {"kind": "box", "box_lo": (0.0, 0.0, 0.0), "box_hi": (1.0, 1.0, 1.0),
            "data_kind": "sources", "quad": [0.0] * 10, "src": cube_sources(seed),
            "holes": np.zeros((0, 6)), "eps": eps, "max_steps": max_steps}


# ----------------------------------------------------------------- patches


def _empty_patches(P):
    return {"c": np.zeros((P, 3)), "n": np.zeros((P, 3)), "t1": np.zeros((P, 3)),
            "h": np.zeros(P), "n_theta": np.zeros(P, np.int32), "n_phi": np.zeros(P, np.int32),
            "n_rings": np.zeros(P, np.int32), "n_sectors": np.zeros(P, np.int32)}


def patches_ball_pole(h=0.2, n_theta=8, n_phi=16, n_rings=4, n_sectors=8):
    """One patch at the north pole of the unit ball; t1 = e_x there."""
    p = _empty_patches(1)
    p["c"][0] = (0.0, 0.0, 1.0)
    p["n"][0] = (0.0, 0.0, 1.0)
    p["t1"][0] = (1.0, 0.0, 0.0)
    p["h"][0] = h
    p["n_theta"][0], p["n_phi"][0], p["n_rings"][0], p["n_sectors"][0] = n_theta, n_phi, n_rings, n_sectors
    return p


def patches_cube_tiles(m=16, n_theta=16, n_phi=32, n_rings=4, n_sectors=16, lo=0.0, hi=1.0):
    """Each face of the box [lo,hi]^3 split into m x m square tiles; one patch
    per tile, centred on it, with h = half the tile side.

    Face order -x,+x,-y,+y,-z,+z; on the face with normal +-e_k the tangent is
    t1 = e_{(k+1) mod 3}; tiles run with the (k+1) coordinate major."""
    side = (hi - lo) / m
    P = 6 * m * m
    p = _empty_patches(P)
    idx = 0
    for face in range(6):
        k = face // 2
        sgn = 1.0 if face % 2 else -1.0
        a, b = (k + 1) % 3, (k + 2) % 3
        for i in range(m):
            for j in range(m):
                c = np.zeros(3)
                c[k] = hi if sgn > 0 else lo
                c[a] = lo + (i + 0.5) * side
                c[b] = lo + (j + 0.5) * side
                n = np.zeros(3)
                n[k] = sgn
                t1 = np.zeros(3)
                t1[a] = 1.0
                p["c"][idx], p["n"][idx], p["t1"][idx] = c, n, t1
                idx += 1
    p["h"][:] = 0.5 * side
    p["n_theta"][:], p["n_phi"][:], p["n_rings"][:], p["n_sectors"][:] = n_theta, n_phi, n_rings, n_sectors
    return p


def subset_patches(p, idx):
    idx = np.asarray(idx)
    return {k: np.ascontiguousarray(v[idx]) for k, v in p.items()}


def cube_tile_subset(m=16, seed=16):
    """A fixed 16-tile sample of the m x m cube tiling: 4 face centres, 4 edge
    tiles, 4 corner tiles and 4 seeded random tiles (indices into
    patches_cube_tiles)."""
    def tid(face, i, j):
        return face * m * m + i * m + j
    c = m // 2
    idx = [tid(0, c, c), tid(1, c - 1, c), tid(2, c, c - 1), tid(5, c - 1, c - 1),
           tid(0, 0, c), tid(3, m - 1, c), tid(4, c, 0), tid(1, c, m - 1),
           tid(0, 0, 0), tid(1, m - 1, m - 1), tid(2, 0, m - 1), tid(5, m - 1, 0)]
    rng = np.random.default_rng(seed)
    rest = [t for t in rng.permutation(6 * m * m) if t not in idx][:4]
    return np.array(idx + [int(t) for t in rest], dtype=np.int64)


# ------------------------------------------------------------------ points


def interior_points_box(n, seed, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0), margin=0.0):
    rng = np.random.default_rng(seed)
    lo = np.asarray(lo) + margin
    hi = np.asarray(hi) - margin
    return lo + rng.random((n, 3)) * (hi - lo)


def interior_points_ball(n, seed, r_max=0.99):
    rng = np.random.default_rng(seed)
    d = rng.standard_normal((n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    r = r_max * rng.random(n) ** (1.0 / 3.0)
    return d * r[:, None]


def cube_targets(n=10_000, seed=2):
    """Potential evaluation targets uniform in the unit cube (own stream)."""
    rng = np.random.default_rng([seed, 1])
    return rng.random((n, 3))


# ----------------------------------------------------------------- configs

CONFIGS = {
    "ball_pole": {  # unit ball, one patch, FP64
        "geometry": geometry_ball_quadratic,
        "patches": patches_ball_pole,
        "walks": 10_000,
        "seed": 1,
    },
    "cube_1536": {  # unit cube, 6 x 16 x 16 patches, FP64
        "geometry": geometry_cube_sources,
        "patches": patches_cube_tiles,
        "walks": 100_000,
        "seed": 2,
        "targets": cube_targets,
    },
}
