"""Shared test helpers: build the oracle for a case dict of `workloads`, and
compare GPU fields with oracle fields."""
import numpy as np

from oracle import diagnostics as odiag
from oracle.model import Oracle, Params, beta_kappa


def oracle_for(c, **over):
    beta, kappa = beta_kappa(c["sigma"], c["width"])
    kw = dict(lattice=c["lattice"], shape=tuple(c["shape"]), periodic=tuple(c["periodic"]),
              tau=c.get("tau", 0.8), mobility=c.get("mobility", 0.1), beta=beta, kappa=kappa,
              rho_l=c.get("rho_l", 10.0), rho_g=c.get("rho_g", 1.0), theta_deg=c["theta_deg"],
              phase_lattice=c.get("phase_lattice", ""), chi_case=c.get("chi_case", 2))
    kw.update(over)
    return Oracle(Params(**kw), c["mask"], c["phi0"])


def oracle_theta(o, c, fields=None):
    f = fields if fields is not None else o.fields()
    return odiag.contact_angle(f["phi"], o.domain(o.zeta), c["wall"], c["width"])


def maxdiff(a, b, mask=None):
    d = np.abs(np.asarray(a) - np.asarray(b))
    if mask is not None:
        d = d[mask]
    return float(d.max()) if d.size else 0.0
