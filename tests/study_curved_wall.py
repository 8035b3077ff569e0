"""Study of the contact-angle deficit on a curved wall (Sec. 3.3), in the oracle
only (CPU; not collected by pytest, run as a script).

On the Sec. 3.3 cylinder the library and the oracle settle a 120 deg drop near
115 deg.  Two readings of the paper could move that:

  axis   -- the boundary-node set of Sec. 2.2.2 built from the axis links only
            (a solid node is a boundary node when a fluid node is one axis step
            away), instead of every lattice link (reading R8, the method);
  smooth -- a_v of Eq. (avvv) from the fluid area fraction of each cell against
            the exact circle, instead of the 0/1 staircase epsilon.

Each run starts from the cap of radius R that meets the wall circle at theta
(the method's equilibrium shape up to the interface profile) and reports theta
every `every` steps, so the direction and size of the drift show where the
reading's equilibrium lies.  Readings are swapped in by replacing the oracle's
module-level classify / effective_area in this process only.

    python tests/study_curved_wall.py [--n 96] [--steps 60000] [--jobs 4]
"""
import argparse
import json
import math
import multiprocessing as mp
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def _cap_case(theta, n, width, mobility):
    import numpy as np
    import workloads
    c = workloads.sec33_cylinder_case(theta, width=width, n=n)
    k = n / 256.0
    rs, centre = 60.0 * k, (n / 2.0, n / 2.0 - 50.0 * k)
    wall = c["wall"]
    r = 50.0 * k * 0.6
    cc = workloads._cap_centre(wall, None, r, theta)
    c["phi0"] = np.ascontiguousarray(workloads.droplet((n, n), cc, r, width), dtype=np.float64)
    c["mobility"] = mobility
    return c, rs, centre


def _run(job):
    variant, theta, n, steps, every, width, mobility = job
    import numpy as np
    import oracle.model as om
    from oracle import diagnostics as od
    from tests.helpers import oracle_for

    c, rs, centre = _cap_case(theta, n, width, mobility)
    base_classify, base_area = om.classify, om.effective_area

    def classify_axis(grid, L, solid_mask):
        zeta, eps, ghost, boundary = base_classify(grid, L, solid_mask)
        solid = grid.from_domain(np.asarray(solid_mask, dtype=bool), fill=True)
        fluid = grid.inside & ~solid
        near = np.zeros(grid.N, dtype=bool)
        for i in range(1, L.Q):
            if int((L.c[i] ** 2).sum()) != 1:
                continue
            nb, ok = grid.shift(L.c[i])
            near |= ok & fluid[nb]
        boundary = grid.inside & solid & near
        zeta = fluid | boundary
        ghost = np.zeros(grid.N, dtype=bool)
        for i in range(1, L.Q):
            nb, ok = grid.shift(L.c[i])
            ghost |= ok & zeta[nb]
        ghost &= ~zeta
        return zeta, eps, ghost, boundary

    def area_smooth(grid, L, eps, zeta):
        # fluid area fraction of each domain cell outside the circle of radius
        # rs about `centre` (the mask's geometric solid), 16 x 16 samples a cell
        sub = (np.arange(16) + 0.5) / 16.0 - 0.5
        nx, ny = c["shape"]
        xs = np.arange(nx)[:, None, None, None] + sub[None, None, :, None]
        ys = np.arange(ny)[None, :, None, None] + sub[None, None, None, :]
        inside = (xs - centre[0]) ** 2 + (ys - centre[1]) ** 2 <= rs * rs
        frac = 1.0 - inside.mean(axis=(2, 3))          # (nx, ny)
        e = grid.from_domain(frac.T, fill=0)
        g = om.gradient(grid, L, e)
        return np.where(zeta, np.sqrt((g ** 2).sum(axis=0)), 0.0)

    if variant in ("axis", "axis+smooth"):
        om.classify = classify_axis
    if variant in ("smooth", "axis+smooth"):
        om.effective_area = area_smooth
    o = oracle_for(c)
    om.classify, om.effective_area = base_classify, base_area
    hist = []
    for t in range(0, steps + 1, every):
        if t:
            o.step(every)
        f = o.fields()
        zeta = o.domain(o.zeta).astype(bool)
        th = od.contact_angle(f["phi"], zeta, c["wall"], c["width"])[0]
        hist.append((t, round(float(th), 3)))
    return dict(variant=variant, theta=theta, n=n, width=width, mobility=mobility, history=hist)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=96)
    ap.add_argument("--steps", type=int, default=60000)
    ap.add_argument("--every", type=int, default=5000)
    ap.add_argument("--width", type=float, default=4.0)
    ap.add_argument("--mobility", type=float, default=0.1)
    ap.add_argument("--thetas", default="120,60")
    ap.add_argument("--variants", default="method,axis,smooth,axis+smooth")
    ap.add_argument("--jobs", type=int, default=4)
    a = ap.parse_args()
    jobs = [(v, float(t), a.n, a.steps, a.every, a.width, a.mobility)
            for t in a.thetas.split(",") for v in a.variants.split(",")]
    with mp.get_context("spawn").Pool(a.jobs) as pool:
        for r in pool.imap_unordered(_run, jobs):
            print(json.dumps(r), flush=True)


if __name__ == "__main__":
    main()
