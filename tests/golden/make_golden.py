"""Writes the stored oracle results used by the GPU parity tests.

    python tests/golden/make_golden.py

Calls only the oracle (and the seeded input generators); nothing here touches
the GPU library.
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads  # noqa: E402
from oracle import diagnostics as odiag  # noqa: E402
from oracle.model import Oracle, Params, beta_kappa  # noqa: E402


def flat_128x64_fp64(steps=5000, every=100):
    c = workloads.flat_128x64_fp64()
    beta, kappa = beta_kappa(c["sigma"], c["width"])
    o = Oracle(Params(lattice="D2Q9", shape=c["shape"], periodic=c["periodic"], tau=0.8,
                      mobility=0.1, beta=beta, kappa=kappa, rho_l=10.0, rho_g=1.0,
                      theta_deg=c["theta_deg"]), c["mask"], c["phi0"])
    mass = [o.mass()]
    for k in range(steps // every):
        o.step(every)
        mass.append(o.mass())
    f = o.fields()
    theta, centre, radius, npts = odiag.contact_angle(f["phi"], o.domain(o.zeta), c["wall"],
                                                      c["width"])
    np.savez_compressed(os.path.join(HERE, "flat_128x64_fp64.npz"), phi=f["phi"], p=f["p"],
                        u=f["u"], mu=f["mu"], mass=np.array(mass), mass_every=every,
                        steps=steps, theta=theta, radius=radius, centre=centre)
    print(f"flat 128x64 FP64: theta {theta:.4f} deg, R {radius:.4f}, points {npts}, mass {mass[-1]:.12f}")


if __name__ == "__main__":
    flat_128x64_fp64()
