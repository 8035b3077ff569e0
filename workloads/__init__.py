"""Seeded synthetic inputs: solid masks, initial order-parameter fields and case
samplers.  Shared by the tests, the benchmark and the smoke check; holds none of
the solver's arithmetic.

Arrays use numpy shape (ny, nx) in 2D and (nz, ny, nx) in 3D, i.e. x is the
fastest index once flattened.  A mask entry is 1 on geometric solid nodes.

The geometries follow the paper's test problems (Sec. 3): a droplet resting on a
flat wall (Sec. 3.1), on an inclined wall built as a staircase (Sec. 3.2) and on
a cylinder or sphere (Sec. 3.3); the initial field is the tanh droplet of Eq.
(initialphi).  Each case also records the wall it rests on (a plane, or a circle
or sphere), which the contact-angle estimators need.

Where the wall is.  A node-centred mask puts the geometric surface half a node
outside its outermost solid nodes.  Those outermost solid nodes become boundary
nodes that carry populations, so the bounce-back wall and the mirror plane of
the zero-gradient ghost condition lie one node further in: half-way between the
boundary nodes and the ghost nodes.  The recorded wall is that plane (the
geometric surface moved one node into the solid), and droplets are centred on
it.
"""
import math

import numpy as np


# ---------------------------------------------------------------- geometry

def _grid(shape):
    """Coordinate arrays (x, y[, z]) over numpy shape reversed(shape)."""
    axes = [np.arange(n, dtype=np.float64) for n in shape]
    mesh = np.meshgrid(*axes[::-1], indexing="ij")
    return mesh[::-1]


def flat_walls(shape, bottom=True, top=True):
    """Solid rows at the lowest (y, or z in 3D) index and/or the highest."""
    mask = np.zeros(shape[::-1], dtype=np.uint8)
    if len(shape) == 2:
        if bottom:
            mask[0, :] = 1
        if top:
            mask[-1, :] = 1
    else:
        if bottom:
            mask[0, :, :] = 1
        if top:
            mask[-1, :, :] = 1
    return mask


def inclined_plane(shape, point, angle_deg):
    """Staircase solid below a plane tilted by angle_deg about the y axis
    (3D: solid where (z - zp) cos a - (x - xp) sin a < 0) or, in 2D, below the line
    through point with slope tan(a) (solid where (y - yp) cos a - (x - xp) sin a < 0)."""
    a = math.radians(angle_deg)
    X = _grid(shape)
    up = X[-1] if len(shape) == 3 else X[1]
    level = (up - point[1]) * math.cos(a) - (X[0] - point[0]) * math.sin(a)
    return (level < 0).astype(np.uint8)


def ball(shape, center, radius):
    """Solid disc (2D) or sphere (3D): nodes strictly inside the radius."""
    X = _grid(shape)
    r2 = sum((X[d] - center[d]) ** 2 for d in range(len(shape)))
    return (r2 < radius * radius).astype(np.uint8)


def droplet(shape, center, radius, width):
    """Eq. (initialphi): 0.5 + 0.5 tanh(2 (R - |x - x0|) / W)."""
    X = _grid(shape)
    r = np.sqrt(sum((X[d] - center[d]) ** 2 for d in range(len(shape))))
    return 0.5 + 0.5 * np.tanh(2.0 * (radius - r) / width)


# ---------------------------------------------------------------- cases

def _case(lattice, shape, periodic, mask, phi0, theta, sigma, width, wall, **kw):
    d = dict(lattice=lattice, shape=tuple(shape), periodic=tuple(periodic),
             mask=np.ascontiguousarray(mask, dtype=np.uint8),
             phi0=np.ascontiguousarray(phi0, dtype=np.float64),
             theta_deg=float(theta), sigma=float(sigma), width=float(width),
             tau=0.8, mobility=0.1, rho_l=10.0, rho_g=1.0, wall=wall)
    d.update(kw)
    return d


def flat_droplet_case(nx=128, ny=64, radius=20.0, theta=60.0, width=4.0,
                      sigma=1e-3, lattice="D2Q9"):
    """Droplet centred on a flat bottom wall; one solid row at the bottom and at
    the top; periodic in x.  The solid row y = 0 holds the boundary nodes, so the
    wall plane is y = -0.5."""
    shape = (nx, ny)
    mask = flat_walls(shape)
    phi0 = droplet(shape, (nx / 2, -0.5), radius, width)
    wall = dict(kind="plane", point=(0.0, -0.5), normal=(0.0, 1.0))
    return _case(lattice, shape, (True, False), mask, phi0, theta, sigma, width, wall)


def flat_cap_case(nx=128, ny=64, radius=20.0, theta=60.0, width=4.0, sigma=1e-3):
    """As flat_droplet_case, but the circle of `radius` is placed so that it
    meets the wall plane y = -0.5 at theta (the equilibrium shape up to the
    interface profile) instead of being centred on it."""
    c = flat_droplet_case(nx, ny, radius, theta, width, sigma)
    centre = _cap_centre(c["wall"], (nx / 2.0, -0.5), radius, theta)
    c["phi0"] = np.ascontiguousarray(droplet((nx, ny), centre, radius, width), dtype=np.float64)
    return c


def flat_128x64_fp64():
    """128 x 64 D2Q9, FP64, R = 20, theta = 60 deg, W = 4, sigma = 1e-3, 5000 steps."""
    c = flat_droplet_case(128, 64, 20.0, 60.0, 4.0)
    c.update(storage="f64", steps=5000, name="flat-128x64-fp64")
    return c


def flat_1024x512_fp32(theta=60.0, nx=1024, ny=512):
    """1024 x 512 D2Q9, FP32, R = 80 on a flat wall, W = 5; 50k steps."""
    c = flat_droplet_case(nx, ny, 80.0 * nx / 1024, theta, 5.0)
    c.update(storage="f32", steps=50000, name=f"flat-{nx}x{ny}-fp32-theta{int(theta)}")
    return c


def inclined_droplet_case_3d(n=256, radius=40.0, theta=45.0, angle=30.0, width=5.0,
                             sigma=1e-3, storage="f32"):
    """n^3 D3Q19, non-periodic; staircase solid below a plane tilted by `angle`
    through (n/2, n/4) in the x-z plane; droplet centred on the wall plane (that
    plane moved one node into the solid)."""
    shape = (n, n, n)
    xp, zp = n / 2.0, n / 4.0
    mask = inclined_plane(shape, (xp, zp), angle)
    a = math.radians(angle)
    nrm = (-math.sin(a), 0.0, math.cos(a))
    c0 = (xp - nrm[0], n / 2.0, zp - nrm[2])
    phi0 = droplet(shape, c0, radius, width)
    wall = dict(kind="plane", point=c0, normal=nrm)
    return _case("D3Q19", shape, (False, False, False), mask, phi0, theta, sigma, width,
                 wall, storage=storage, steps=20000,
                 name=f"inclined-{n}^3-{storage}")


def inclined_3d_256(storage="f32", n=256):
    return inclined_droplet_case_3d(n=n, radius=40.0 * n / 256, storage=storage)


def cylinder_case(nx, ny, rc_frac, theta, width=4.0, sigma=1e-3, drop_frac=0.3):
    """Solid cylinder of radius rc_frac*ny near the bottom, droplet of radius
    drop_frac*R_c centred on its top; walls at the bottom and top rows.  The
    wall circle has radius R_c - 1."""
    rc = rc_frac * ny
    center = (nx / 2.0, rc + 0.05 * ny)
    mask = np.maximum(ball((nx, ny), center, rc), flat_walls((nx, ny)))
    rd = drop_frac * rc
    phi0 = droplet((nx, ny), (center[0], center[1] + rc - 1.0), rd, width)
    wall = dict(kind="circle", center=center, radius=rc - 1.0)
    return _case("D2Q9", (nx, ny), (True, False), mask, phi0, theta, sigma, width, wall,
                 storage="f32", name=f"cyl-{nx}x{ny}")


def table1_case_3d(theta, n=(256, 256, 128), start="centred"):
    """The 3D flat-plate test of Sec. 3.1: Nx x Ny x Nz, periodic on every side,
    D3Q19 FP32; the plate as in 2D (0.25 Nz thick, 0.05 Nz above the bottom) and
    a drop of R = 50 (scaled with Nz / 128) centred at (Nx/2, Ny/2, 0.25 Nz), the
    centre the paper prints; rows below the plate's top row start dry.  The wall
    plane of the angle fit is half a node below the plate's top row.
    start="cap": the sphere of the same R placed so that it meets that plane at
    theta (the equilibrium shape up to the interface profile)."""
    nx, ny, nz = n
    z_lo, thick = round(0.05 * nz), round(0.25 * nz)
    mask = np.zeros((nz, ny, nx), dtype=np.uint8)
    mask[z_lo:z_lo + thick] = 1
    z_wall = z_lo + thick - 1.5
    R = {10.0: 30.0, 20.0: 40.0}.get(float(theta), 50.0) * nz / 128.0
    centre = (nx / 2.0, ny / 2.0, 0.25 * nz)
    if start == "cap":
        centre = (nx / 2.0, ny / 2.0, z_wall - R * math.cos(math.radians(theta)))
    phi0 = droplet(n, centre, R, 4.0)
    phi0[:z_lo + thick - 1] = 0.0
    wall = dict(kind="plane", point=(0.0, 0.0, z_wall), normal=(0.0, 0.0, 1.0))
    c = _case("D3Q19", n, (True, True, True), mask, phi0, theta, 0.005, 4.0, wall)
    c.update(mobility=0.01, storage="f32", radius=R, name=f"table1-3d-{int(theta)}")
    return c


SEC32_SLOPES = (1.0, 0.5, 0.25)
SEC3_ANGLES = (30.0, 60.0, 90.0, 120.0, 150.0)


def sec32_incline_case(theta, slope, width=4.0, n=256):
    """Sec. 3.2 in 2D: an n x n box, closed on all sides, solid below the line
    y = slope x; a semicircular drop of R = 50 (scaled with n) centred on the
    line at x = n/2.  The wall the angle is measured against is that line moved
    one node into the solid along its normal (the bounce-back plane of flat
    walls).  sigma = 0.005, M = 0.01, rho 10/1, nu 0.1 in both phases."""
    shape = (n, n)
    gam = math.atan(slope)
    mask = inclined_plane(shape, (0.0, 0.0), math.degrees(gam))
    nrm = (-math.sin(gam), math.cos(gam))
    x0 = n / 2.0
    R = 50.0 * n / 256.0
    # the lower half of the circle lies in the solid, where only the boundary
    # nodes (zeta = 1) read it
    phi0 = droplet(shape, (x0, slope * x0), R, width)
    wall = dict(kind="plane", point=(-nrm[0], -nrm[1]), normal=nrm)
    c = _case("D2Q9", shape, (False, False), mask, phi0, theta, 0.005, width, wall)
    c.update(mobility=0.01, storage="f32", radius=R,
             name=f"sec32-slope{slope}-theta{int(theta)}-W{int(width)}")
    return c


def sec32_incline_case_3d(theta, slope, n=256, width=6.0, start="paper"):
    """Sec. 3.2 in 3D: an n^3 box, closed on all sides, solid below the plane
    z = slope x; a drop of R = 50 (scaled with n / 256) centred on the plane at
    (n/2, n/2, slope n/2).  The wall the angle is measured against is that plane
    moved one node into the solid along its normal.  start="cap": the sphere of
    the same R placed so that it meets that wall at theta.  sigma = 0.005,
    M = 0.01, rho 10/1, nu 0.1 in both phases, W = 6, D3Q19 FP32."""
    shape = (n, n, n)
    gam = math.atan(slope)
    mask = inclined_plane(shape, (0.0, 0.0), math.degrees(gam))
    nrm = (-math.sin(gam), 0.0, math.cos(gam))
    x0 = n / 2.0
    R = 50.0 * n / 256.0
    wall = dict(kind="plane", point=(-nrm[0], 0.0, -nrm[2]), normal=nrm)
    centre = (x0, n / 2.0, slope * x0)
    if start == "cap":
        foot = tuple(centre[k] - nrm[k] for k in range(3))
        centre = _cap_centre(wall, foot, R, theta)
    phi0 = droplet(shape, centre, R, width)
    c = _case("D3Q19", shape, (False, False, False), mask, phi0, theta, 0.005, width, wall)
    c.update(mobility=0.01, storage="f32", radius=R,
             name=f"sec32-3d-slope{slope}-theta{int(theta)}")
    return c


def sec33_cylinder_case(theta, width=6.0, n=256, start="paper"):
    """Sec. 3.3 in 2D: a solid cylinder of radius R_s = 60 centred at
    (n/2, n/2 - 50) in an n x n box (scaled with n), periodic in x and closed in
    y; a drop of R_i = 50 centred at (n/2, n/2), inside the cylinder's top (only
    zeta = 1 nodes read phi0).  The wall circle of the angle fit has radius
    R_s - 1.  start="cap": instead, a circle of radius 0.6 R_i placed so that
    it meets the wall circle at theta (the equilibrium shape up to the interface
    profile), so the contact line need not travel over the staircase.
    sigma = 0.005, M = 0.01, rho 10/1, nu 0.1 in both phases, W = 6."""
    shape = (n, n)
    k = n / 256.0
    rs, centre = 60.0 * k, (n / 2.0, n / 2.0 - 50.0 * k)
    mask = ball(shape, centre, rs)
    wall = dict(kind="circle", center=centre, radius=rs - 1.0)
    if start == "cap":
        r = 0.6 * 50.0 * k
        phi0 = droplet(shape, _cap_centre(wall, None, r, theta), r, width)
    else:
        phi0 = droplet(shape, (n / 2.0, n / 2.0), 50.0 * k, width)
    c = _case("D2Q9", shape, (True, False), mask, phi0, theta, 0.005, width, wall)
    c.update(mobility=0.01, storage="f32", name=f"sec33-cylinder-theta{int(theta)}")
    return c


def sec33_sphere_case(theta, n=256, width=6.0, start="paper"):
    """Sec. 3.3 in 3D: a solid sphere of radius R_s = 60 centred at
    (n/2, n/2, n/2 - 50) in an n^3 box (scaled with n / 256), periodic in x and
    y and closed in z; a drop of R_i = 50 centred at (n/2, n/2, n/2).  The wall
    sphere of the angle fit has radius R_s - 1.  start="cap": a sphere of radius
    0.6 R_i placed so that it meets the wall sphere at theta.  sigma = 0.005, M = 0.01,
    rho 10/1, nu 0.1 in both phases, W = 6, D3Q19 FP32."""
    shape = (n, n, n)
    k = n / 256.0
    rs, centre = 60.0 * k, (n / 2.0, n / 2.0, n / 2.0 - 50.0 * k)
    mask = ball(shape, centre, rs)
    wall = dict(kind="ball", center=centre, radius=rs - 1.0)
    if start == "cap":
        r = 0.6 * 50.0 * k
        phi0 = droplet(shape, _cap_centre(wall, None, r, theta), r, width)
    else:
        phi0 = droplet(shape, (n / 2.0, n / 2.0, n / 2.0), 50.0 * k, width)
    c = _case("D3Q19", shape, (True, True, False), mask, phi0, theta, 0.005, width, wall)
    c.update(mobility=0.01, storage="f32", name=f"sec33-sphere-theta{int(theta)}")
    return c


def cylinder_batch(seed=3, n_cases=64, start="drop"):
    """64 D2Q9 cylinder cases, sizes U{128..768 step 16} x half, R_c ~ U[0.2, 0.4] Ny,
    droplet 0.3 R_c, theta ~ U[30, 150] deg, W = 4, FP32.  start="drop": the
    droplet is centred on the top of the cylinder (it meets the wall at 90
    degrees); start="cap": the same radius placed so that it meets the
    cylinder at its theta (see serving_request)."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n_cases):
        nx = int(rng.integers(0, (768 - 128) // 16 + 1)) * 16 + 128
        ny = nx // 2
        rcf = float(rng.uniform(0.2, 0.4))
        th = float(rng.uniform(30.0, 150.0))
        c = cylinder_case(nx, ny, rcf, th)
        if start == "cap":
            rd = 0.3 * rcf * ny
            c["phi0"] = np.ascontiguousarray(droplet((nx, ny), _cap_centre(c["wall"], None, rd, th),
                                                     rd, c["width"]))
        c["name"] = f"c3-{k:02d}-{nx}x{ny}"
        c["start"] = start
        out.append(c)
    return out


TABLE1_ANGLES = (10.0, 20.0, 30.0, 40.0, 60.0, 90.0, 120.0, 140.0, 150.0, 160.0, 170.0)


def table1_case(theta, nx=256, ny=128):
    """The flat-plate test of Sec. 3.1 (Table 1, 2D): nx x ny, periodic on all
    sides, a solid plate 0.25 ny thick whose bottom lies 0.05 ny above the
    lower edge, a semicircular droplet of radius 50 (40 at 20 deg, 30 at 10 deg)
    centred on the plate's wall plane; rho 10/1, nu 0.1 (tau 0.8), sigma 0.005,
    M 0.01, W 4."""
    y_lo, thick = round(0.05 * ny), round(0.25 * ny)
    mask = np.zeros((ny, nx), dtype=np.uint8)
    mask[y_lo:y_lo + thick, :] = 1
    y_wall = y_lo + thick - 1.5          # the top solid row moved half a node into the solid
    R = {10.0: 30.0, 20.0: 40.0}.get(float(theta), 50.0) * ny / 128.0
    phi0 = droplet((nx, ny), (nx / 2.0, y_wall), R, 4.0)
    # a semicircle: every row below the plate's top row is cleared, so that the
    # lower half of the circle puts no liquid on the plate's underside boundary
    # nodes or in the gas below the plate
    phi0[:y_lo + thick - 1, :] = 0.0
    wall = dict(kind="plane", point=(0.0, y_wall), normal=(0.0, 1.0))
    c = _case("D2Q9", (nx, ny), (True, True), mask, phi0, theta, 0.005, 4.0, wall)
    c.update(mobility=0.01, storage="f32", radius=R, name=f"table1-{int(theta)}")
    return c


def _cap_centre(wall, foot, radius, theta):
    """Centre of a circle / sphere of `radius` that meets `wall` at the contact
    angle theta (degrees), on the fluid side: for a plane, at signed height
    -R cos(theta) along the normal from `foot`, a point of the plane
    (cos theta = -h / R); for a circle or sphere of radius R_w, at distance
    d = sqrt(R^2 + R_w^2 - 2 R R_w cos theta) from its centre, straight above it
    (cos theta = (R^2 + R_w^2 - d^2) / (2 R R_w))."""
    ct = math.cos(math.radians(theta))
    if wall["kind"] == "plane":
        n = wall["normal"]
        return tuple(foot[k] - radius * ct * n[k] for k in range(len(foot)))
    c, rw = wall["center"], wall["radius"]
    d = math.sqrt(radius * radius + rw * rw - 2.0 * radius * rw * ct)
    up = [0.0] * len(c)
    up[-1] = 1.0
    return tuple(c[k] + d * up[k] for k in range(len(c)))


def serving_request(rng, idx, nx_range=(256, 1024), n3_range=(64, 192), start="drop"):
    """One request of the serving workload: 2D (256x128 .. 1024x512) or 3D
    (64^3 .. 192^3), geometry flat / inclined / curved, theta ~ U[30, 150].

    start="drop": a circle / sphere of R = 0.2 N centred on the wall (it meets
    the wall at 90 degrees and must spread or retract to theta).  start="cap":
    the same radius placed so that it already meets the wall at theta, the
    equilibrium shape of the method up to the interface profile; the request
    then asks for the steady state near that shape."""
    th = float(rng.uniform(30.0, 150.0))
    geom = ["flat", "inclined", "curved"][int(rng.integers(0, 3))]
    if rng.uniform() < 0.5:
        lo, hi = nx_range
        nx = int(rng.integers(0, (hi - lo) // 32 + 1)) * 32 + lo
        ny = nx // 2
        R = 0.2 * ny
        if geom == "flat":
            c = flat_droplet_case(nx, ny, R, th, 5.0)
        elif geom == "inclined":
            a = 30.0
            xp, yp = nx / 2.0, ny / 4.0
            mask = np.maximum(inclined_plane((nx, ny), (xp, yp), a), flat_walls((nx, ny)))
            r = math.radians(a)
            nrm = (-math.sin(r), math.cos(r))
            c0 = (xp - nrm[0], yp - nrm[1])
            phi0 = droplet((nx, ny), c0, R, 5.0)
            wall = dict(kind="plane", point=c0, normal=nrm)
            c = _case("D2Q9", (nx, ny), (True, False), mask, phi0, th, 1e-3, 5.0, wall)
        else:
            c = cylinder_case(nx, ny, 0.3, th, width=5.0, drop_frac=R / (0.3 * ny))
    else:
        lo, hi = n3_range
        n = int(rng.integers(0, (hi - lo) // 16 + 1)) * 16 + lo
        R = 0.2 * n
        shape = (n, n, n)
        if geom == "flat":
            mask = flat_walls(shape, bottom=True, top=False)
            phi0 = droplet(shape, (n / 2, n / 2, -0.5), R, 5.0)
            wall = dict(kind="plane", point=(0.0, 0.0, -0.5), normal=(0.0, 0.0, 1.0))
        elif geom == "inclined":
            c = inclined_droplet_case_3d(n=n, radius=R, theta=th)
            mask, phi0, wall = c["mask"], c["phi0"], c["wall"]
        else:
            rs = 0.3 * n
            center = (n / 2, n / 2, rs + 0.05 * n)
            mask = ball(shape, center, rs)
            phi0 = droplet(shape, (n / 2, n / 2, center[2] + rs - 1.0), R, 5.0)
            wall = dict(kind="circle", center=center, radius=rs - 1.0)
        c = _case("D3Q19", shape, (False, False, False), mask, phi0, th, 1e-3, 5.0, wall)
    if start == "cap":
        sh = c["shape"]
        R = 0.2 * (sh[1] if c["lattice"] == "D2Q9" else sh[0])
        w = c["wall"]
        if w["kind"] == "plane":
            # the drop's foot: the plane's point below the middle of the domain
            mid = np.array([0.5 * v for v in sh], dtype=np.float64)
            p0, nrm = np.asarray(w["point"], float), np.asarray(w["normal"], float)
            foot = tuple(mid - ((mid - p0) @ nrm) * nrm)
        else:
            foot = None
        c["phi0"] = np.ascontiguousarray(droplet(sh, _cap_centre(w, foot, R, th), R, 5.0))
    c.update(storage="f32", geometry=geom, start=start, name=f"req-{idx:03d}-{geom}-{c['lattice']}")
    return c


def serving_requests(seed=4, n_requests=200, rate=20.0, nx_range=(256, 1024), n3_range=(64, 192),
                     start="drop"):
    """Poisson arrivals (mean `rate` per second) of mixed serving requests."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for k in range(n_requests):
        t += float(rng.exponential(1.0 / rate))
        c = serving_request(rng, k, nx_range, n3_range, start=start)
        c["arrival_s"] = t
        out.append(c)
    return out
