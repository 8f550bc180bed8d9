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


def geometry_halfspace_charge(h=1.0, trunc_r=1e5, eps=1e-5, max_steps=1_000_000):
    """Half space z > 0 over a unit charge at (0, 0, -h): u = 1 / |x - s|
    (Sec. 5.1.3, Test 1, eq. bw89 with q'/(4 pi eps0) = 1 and h = 1, the
    constants that give the printed analytic 0.71554).  Walks that reach the
    sphere |x| = trunc_r count as gone to infinity (u = 0 there)."""
    return {"kind": "half_space", "ball_c": (0.0, 0.0, 0.0), "trunc_r": float(trunc_r),
            "data_kind": "sources", "quad": [0.0] * 10, "src": np.array([[0.0, 0.0, -float(h), 1.0]]),
            "holes": np.zeros((0, 6)), "eps": eps, "max_steps": max_steps}


def geometry_disk(b=1.0, trunc_r=1e5, eps=1e-5, max_steps=1_000_000):
    """Exterior of a thin conducting disk {z = 0, x^2 + y^2 <= b^2} held at
    u = 1, with u -> 0 at infinity (Sec. 5.1.3, Test 4, eq. bw95 with Q = 8b);
    walks that reach the sphere |x| = trunc_r count as gone to infinity."""
    return {"kind": "disk", "disk_r": float(b), "ball_c": (0.0, 0.0, 0.0), "trunc_r": float(trunc_r),
            "data_kind": "quadratic", "quad": [1.0] + [0.0] * 9, "src": np.zeros((0, 4)),
            "holes": np.zeros((0, 6)), "eps": eps, "max_steps": max_steps}


# Test 4's point and hemisphere (Sec. 5.1.3) and Table 5's three rules:
# (N_g1, paths per node).
DISK_POINT = {"x": (-0.5, 0.0, 0.0), "n": (0.0, 0.0, -1.0), "t1": (1.0, 0.0, 0.0), "a": 0.4}
TABLE5_RULES = [(10, 100), (10, 1000), (20, 1000)]


def disk_points(n, seed=8, b=1.0, rho_max=0.8, a_max=0.4):
    """Single-point queries on both faces of the disk: centres uniform by area
    in the disk of radius rho_max*b, alternately on the upper face (outward
    normal (0, 0, -1)) and the lower one ((0, 0, 1)), tangent at a uniform
    angle, hemisphere radius a = min(a_max, 0.9 (b - rho)) so that S_a stays
    on the disk.  Rows: x [n,3], normal [n,3], t1 [n,3], a [n]."""
    rng = np.random.default_rng([seed, 19])
    r = rho_max * b * np.sqrt(rng.random(n))
    ang = 2 * np.pi * rng.random(n)
    x = np.column_stack([r * np.cos(ang), r * np.sin(ang), np.zeros(n)])
    nrm = np.zeros((n, 3))
    nrm[:, 2] = np.where(np.arange(n) % 2 == 0, -1.0, 1.0)
    c = 2 * np.pi * rng.random(n)
    t1 = np.column_stack([np.cos(c), np.sin(c), np.zeros(n)])
    a = np.minimum(a_max, 0.9 * (b - r))
    return x, nrm, t1, a


def geometry_ball_exterior(R=3.0, q=1.0, trunc_r=1e5, eps=1e-5, max_steps=1_000_000):
    """Exterior of the sphere |x| = R with a point charge q at its centre,
    u = q/|x| (Sec. 5.2, the big sphere: R = 3, q = 1); walks that reach the
    sphere |x| = trunc_r count as gone to infinity."""
    return {"kind": "ball_exterior", "ball_c": (0.0, 0.0, 0.0), "ball_r": float(R), "trunc_r": float(trunc_r),
            "data_kind": "sources", "quad": [0.0] * 10, "src": np.array([[0.0, 0.0, 0.0, float(q)]]),
            "holes": np.zeros((0, 6)), "eps": eps, "max_steps": max_steps}


def patches_big_sphere(R=3.0, h=1.0, n_theta=16, n_phi=32, n_rings=4, n_sectors=16):
    """Sec. 5.2's patch: centre o = (0, 0, R) on the sphere, a = h = 1; the
    domain's outward normal there points to the centre."""
    d = _empty_patches(1)
    d["c"][0] = (0.0, 0.0, R)
    d["n"][0] = (0.0, 0.0, -1.0)
    d["t1"][0] = (1.0, 0.0, 0.0)
    d["h"][0] = h
    d["n_theta"][0], d["n_phi"][0], d["n_rings"][0], d["n_sectors"][0] = n_theta, n_phi, n_rings, n_sectors
    return d


def patches_sphere_exterior(n, R=3.0, h=0.5, n_theta=8, n_phi=16, n_rings=4, n_sectors=8, seed=9):
    """n patches outside the sphere |x| = R at the points of a Fibonacci
    lattice (near-uniform), each with the domain's outward normal (to the
    centre) and a tangent at a seeded angle."""
    rng = np.random.default_rng([seed, 23])
    k = np.arange(n) + 0.5
    z = 1.0 - 2.0 * k / n
    phi = np.pi * (1.0 + 5.0 ** 0.5) * k
    u = np.column_stack([np.sqrt(1 - z * z) * np.cos(phi), np.sqrt(1 - z * z) * np.sin(phi), z])
    d = _empty_patches(n)
    d["c"][:] = R * u
    d["n"][:] = -u
    ref = np.where(np.abs(u[:, 2:3]) < 0.9, [[0.0, 0.0, 1.0]], [[1.0, 0.0, 0.0]])
    e1 = np.cross(ref, u)
    e1 /= np.linalg.norm(e1, axis=1, keepdims=True)
    e2 = np.cross(u, e1)
    ang = 2 * np.pi * rng.random(n)
    d["t1"][:] = np.cos(ang)[:, None] * e1 + np.sin(ang)[:, None] * e2
    d["h"][:] = h
    d["n_theta"][:], d["n_phi"][:], d["n_rings"][:], d["n_sectors"][:] = n_theta, n_phi, n_rings, n_sectors
    return d


def box_face_grid(gd, n0, n1):
    """Grid points of the six faces of a box geometry (-x,+x,-y,+y,-z,+z),
    face k's axes a = (k+1) mod 3 with n0 nodes and b = (k+2) mod 3 with n1,
    uniform from lo to hi: [6][n0][n1][3]."""
    lo, hi = np.asarray(gd["box_lo"], float), np.asarray(gd["box_hi"], float)
    out = np.zeros((6, n0, n1, 3))
    for f in range(6):
        k, a, b = f // 2, (f // 2 + 1) % 3, (f // 2 + 2) % 3
        A, B = np.meshgrid(np.linspace(lo[a], hi[a], n0), np.linspace(lo[b], hi[b], n1), indexing="ij")
        out[f, :, :, k] = hi[k] if f % 2 else lo[k]
        out[f, :, :, a] = A
        out[f, :, :, b] = B
    return out


def tabulated_cube_sources(n0=257, n1=257, seed=2, eps=1e-5, max_steps=1_000_000):
    """The unit cube with its 8-source data given as face tables (the
    potential sampled on each face's grid): Dirichlet data without a closed
    form for the library, whose harmonic extension approaches the sources'
    potential as the grid is refined (bilinear interpolation error
    O(grid spacing^2))."""
    gd = geometry_cube_sources(seed, eps, max_steps)
    X = box_face_grid(gd, n0, n1)
    src = gd["src"]
    tab = sum(q[3] / np.linalg.norm(X - q[:3], axis=-1) for q in src)
    return dict(gd, data_kind="table", tab=np.ascontiguousarray(tab))


def halfspace_points(n, seed=6, radii=(0.1, 0.2, 0.5, 0.7, 1.0), extent=2.0):
    """Single-point queries on the plane z = 0: points uniform in the disk of
    radius ``extent`` around the origin, hemisphere radius cycling through
    ``radii`` (Table 1's), tangent at a uniform angle.  Rows: x [n,3],
    outward normal [n,3] = (0, 0, -1), t1 [n,3], a [n]."""
    rng = np.random.default_rng([seed, 17])
    r = extent * np.sqrt(rng.random(n))
    ang = 2 * np.pi * rng.random(n)
    x = np.column_stack([r * np.cos(ang), r * np.sin(ang), np.zeros(n)])
    nrm = np.tile([0.0, 0.0, -1.0], (n, 1))
    b = 2 * np.pi * rng.random(n)
    t1 = np.column_stack([np.cos(b), np.sin(b), np.zeros(n)])
    a = np.asarray(radii, float)[np.arange(n) % len(radii)]
    return x, nrm, t1, a


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


# ----------------------------------------------- box minus holes (uneven batches)


def box_holes(seed=4, n_holes=20, size=4.0, side=(0.2, 0.8), gap=0.1, max_tries=100_000):
    """Axis-aligned holes in the box [0,size]^3: independent sides ~U(side),
    placed by rejection at least `gap` from the outer box and separated from
    every other hole by at least `gap` along some axis.  Rows are
    (lo x,y,z, hi x,y,z)."""
    rng = np.random.default_rng(seed)
    holes = []
    tries = 0
    while len(holes) < n_holes:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("could not place the holes")
        e = rng.uniform(side[0], side[1], size=3)
        lo = gap + rng.random(3) * (size - 2 * gap - e)
        hi = lo + e
        ok = True
        for h in holes:
            if not (np.any(lo >= h[3:] + gap) or np.any(hi <= h[:3] - gap)):
                ok = False
                break
        if ok:
            holes.append(np.concatenate([lo, hi]))
    return np.array(holes)


def hole_sources(holes, seed=4):
    """One source per hole, uniform in the hole's central half (a quarter of
    each side inset), charge ~N(0,1).  Rows are (x, y, z, q)."""
    rng = np.random.default_rng([seed, 7])
    lo, hi = holes[:, :3], holes[:, 3:]
    s = lo + (hi - lo) * (0.25 + 0.5 * rng.random(lo.shape))
    q = rng.standard_normal(len(holes))
    return np.ascontiguousarray(np.column_stack([s, q]))


def geometry_box_holes(seed=4, eps=1e-5, max_steps=1_000_000):
    """[0,4]^3 minus 20 holes, u = sum_i q_i / |x - s_i|, one source in each hole."""
    holes = box_holes(seed)
    return {"kind": "box_minus_boxes", "box_lo": (0.0, 0.0, 0.0), "box_hi": (4.0, 4.0, 4.0),
            "data_kind": "sources", "quad": [0.0] * 10, "src": hole_sources(holes, seed),
            "holes": holes, "eps": eps, "max_steps": max_steps}


# panel classes: panels -> (n_theta, n_phi, n_rings, n_sectors)
PANEL_CLASSES = {8: (4, 8, 2, 4), 16: (6, 12, 2, 8), 32: (8, 16, 4, 8), 64: (16, 32, 4, 16), 128: (16, 32, 8, 16)}


def _box_point_dist(c, lo, hi):
    q = np.maximum(np.maximum(lo - c, 0.0), c - hi)
    return float(np.sqrt(np.sum(q * q)))


def patches_box_holes(gd, alpha=0.145, panels_per_area=4000.0):
    """Tiles over every face of the outer box and of the holes, one patch per
    tile.  Patch sizes follow the face areas: a face of sides a x b is split
    into round(a/s) x round(b/s) tiles with s = alpha sqrt(ab), so small hole
    faces get small patches and the large outer faces large ones.  Each patch
    is centred on its tile with h = the smallest of half the shorter tile
    side, the distance to the face's edges and the clearance to every other
    surface (so each half ball stays in the domain).  Panels follow the tile
    area (panels_per_area per unit area), rounded to a class in
    {8, 16, 32, 64, 128}."""
    lo_b, hi_b = np.asarray(gd["box_lo"], float), np.asarray(gd["box_hi"], float)
    holes = np.asarray(gd["holes"], float).reshape(-1, 6)
    faces = []  # (axis, plane, sign of the outward normal of the domain, rect lo, rect hi, owner)
    for k in range(3):
        for sgn, plane in ((-1.0, lo_b[k]), (1.0, hi_b[k])):
            faces.append((k, plane, sgn, lo_b, hi_b, -1))
    for i, h in enumerate(holes):
        for k in range(3):
            # the domain lies outside the hole: its outward normal points into the hole
            faces.append((k, h[k], 1.0, h[:3], h[3:], i))
            faces.append((k, h[3 + k], -1.0, h[:3], h[3:], i))
    rows = []
    classes = np.array(sorted(PANEL_CLASSES))
    for (k, plane, sgn, rlo, rhi, owner) in faces:
        a, b = (k + 1) % 3, (k + 2) % 3
        la, lb = rhi[a] - rlo[a], rhi[b] - rlo[b]
        tile = alpha * np.sqrt(la * lb)
        na, nb = max(1, int(round(la / tile))), max(1, int(round(lb / tile)))
        da, db = la / na, lb / nb
        for i in range(na):
            for j in range(nb):
                c = np.zeros(3)
                c[k] = plane
                c[a] = rlo[a] + (i + 0.5) * da
                c[b] = rlo[b] + (j + 0.5) * db
                edge = min(c[a] - rlo[a], rhi[a] - c[a], c[b] - rlo[b], rhi[b] - c[b])
                clear = np.inf
                for k2 in range(3):
                    for p2 in (lo_b[k2], hi_b[k2]):
                        if owner == -1 and k2 == k and p2 == plane:
                            continue
                        clear = min(clear, abs(c[k2] - p2))
                for i2, h2 in enumerate(holes):
                    if i2 != owner:
                        clear = min(clear, _box_point_dist(c, h2[:3], h2[3:]))
                h = min(0.5 * min(da, db), edge, clear)
                want = panels_per_area * da * db
                P = int(classes[np.argmin(np.abs(np.log(classes / want)))])
                n = np.zeros(3)
                n[k] = sgn
                t1 = np.zeros(3)
                t1[a] = 1.0
                rows.append((c, n, t1, h, P))
    p = _empty_patches(len(rows))
    for idx, (c, n, t1, h, P) in enumerate(rows):
        p["c"][idx], p["n"][idx], p["t1"][idx], p["h"][idx] = c, n, t1, h
        p["n_theta"][idx], p["n_phi"][idx], p["n_rings"][idx], p["n_sectors"][idx] = PANEL_CLASSES[P]
    return p


def box_holes_sample(pd, per_class=2, seed=4):
    """Seeded sample of patch indices, ``per_class`` from every panel class
    present (for tests that compare against the oracle)."""
    rng = np.random.default_rng([seed, 11])
    P = np.asarray(pd["n_rings"]) * np.asarray(pd["n_sectors"])
    out = []
    for c in sorted(set(P.tolist())):
        idx = np.flatnonzero(P == c)
        out.extend(rng.choice(idx, min(per_class, len(idx)), replace=False).tolist())
    return np.array(sorted(out), dtype=np.int64)


def boundary_faces(gd):
    """Faces of a box (with holes): rows (axis, plane, outward normal sign of
    the domain, rect lo [3], rect hi [3])."""
    lo_b, hi_b = np.asarray(gd["box_lo"], float), np.asarray(gd["box_hi"], float)
    faces = []
    for k in range(3):
        faces.append((k, lo_b[k], -1.0, lo_b, hi_b))
        faces.append((k, hi_b[k], 1.0, lo_b, hi_b))
    for h in np.asarray(gd.get("holes", np.zeros((0, 6))), float).reshape(-1, 6):
        for k in range(3):
            faces.append((k, h[k], 1.0, h[:3], h[3:]))
            faces.append((k, h[3 + k], -1.0, h[:3], h[3:]))
    return faces


def boundary_points(gd, n, rng, edge_gap=1e-4):
    """n points uniform by area on the boundary of a box (with holes), with
    their outward normals; points within edge_gap of a face edge are redrawn."""
    faces = boundary_faces(gd)
    area = np.array([(f[4][(f[0] + 1) % 3] - f[3][(f[0] + 1) % 3]) * (f[4][(f[0] + 2) % 3] - f[3][(f[0] + 2) % 3])
                     for f in faces])
    pts = np.empty((n, 3))
    nrm = np.zeros((n, 3))
    fi = rng.choice(len(faces), n, p=area / area.sum())
    for i, f in enumerate(fi):
        k, plane, sgn, lo, hi = faces[f]
        a, b = (k + 1) % 3, (k + 2) % 3
        while True:
            u = rng.random(2)
            pa = lo[a] + u[0] * (hi[a] - lo[a])
            pb = lo[b] + u[1] * (hi[b] - lo[b])
            if min(pa - lo[a], hi[a] - pa, pb - lo[b], hi[b] - pb) > edge_gap:
                break
        pts[i, k], pts[i, a], pts[i, b] = plane, pa, pb
        nrm[i, k] = sgn
    return pts, nrm


def serving_queries(gd, n_queries=600, rate=200.0, seed=5, max_points=4096, se_range=(1e-4, 1e-2)):
    """Poisson arrivals at ``rate`` queries/s; each query has a point count
    log-uniform on [1, max_points], points uniform by area on the boundary
    and a required standard error log-uniform on ``se_range``.  Returns a
    list of dicts (t, pts, normals, se, seed)."""
    rng = np.random.default_rng([seed, 13])
    t = np.cumsum(rng.exponential(1.0 / rate, n_queries))
    lo, hi = np.log(se_range[0]), np.log(se_range[1])
    out = []
    for i in range(n_queries):
        m = int(np.floor(np.exp(rng.random() * np.log(max_points + 1))))
        m = min(max(m, 1), max_points)
        pts, nrm = boundary_points(gd, m, rng)
        se = float(np.exp(lo + (hi - lo) * rng.random()))
        out.append({"t": float(t[i]), "pts": pts, "normals": nrm, "se": se, "seed": int(seed) * 1_000_003 + i})
    return out


# ----------------------------------------------------------------- configs

CONFIGS = {
    "sphere_exterior": {  # Sec. 5.2 scaled: 2048 patches outside the sphere R = 3, 1e4 walks per node
        "geometry": geometry_ball_exterior,
        "patches": patches_sphere_exterior,
        "n_patches": 2048,
        "walks": 10_000,
        "seed": 9,
    },
    "disk_points": {  # Test 4 scaled to many points on both faces: 20x20 nodes, 1e3 walks each
        "geometry": geometry_disk,
        "points": disk_points,
        "n_points": 4096,
        "n_g1": 20,
        "n_g2": 20,
        "delta_rel": 1e-6,
        "walks": 1000,
        "seed": 8,
    },
    "halfspace_points": {  # Test 1 scaled to many points: 20x20 nodes, 1e3 walks each
        "geometry": geometry_halfspace_charge,
        "points": halfspace_points,
        "n_points": 4096,
        "n_g1": 20,
        "n_g2": 20,
        "delta_rel": 1e-6,
        "walks": 1000,
        "seed": 6,
    },
    "ball_pole": {  # unit ball, one patch, FP64
        "geometry": geometry_ball_quadratic,
        "patches": patches_ball_pole,
        "walks": 10_000,
        "seed": 1,
    },
    "box_holes": {  # [0,4]^3 minus 20 holes, ~6000 uneven patches, adaptive walks
        "geometry": geometry_box_holes,
        "patches": patches_box_holes,
        "se_target": 1e-3,
        "pilot_walks": 1000,
        "min_walks": 1000,
        "max_walks": 200_000,
        "seed": 4,
    },
    "serving": {  # box_holes geometry resident, Poisson query arrivals
        "geometry": geometry_box_holes,
        "queries": serving_queries,
        "rate": 200.0,
        "n_queries": 600,
        "se_range": (1e-4, 1e-2),
        "pilot_walks": 100,
        "min_walks": 100,
        "max_walks": 1_000_000,
        "h_max": 0.25,
        "ladder": 16,
        "layout": (8, 16, 4, 8),
        "hbm_budget": 2 << 30,
        "seed": 5,
    },
    "cube_1536": {  # unit cube, 6 x 16 x 16 patches, FP64
        "geometry": geometry_cube_sources,
        "patches": patches_cube_tiles,
        "walks": 100_000,
        "seed": 2,
        "targets": cube_targets,
    },
}
