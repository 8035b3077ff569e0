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
              phase_lattice=c.get("phase_lattice", ""), chi_case=c.get("chi_case", 2),
              theta_map=c.get("theta_map"))
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


def window(c, centre, half):
    """Sub-box of case `c` of half-width `half` around the node `centre`
    ((x, y) or (x, y, z)) as a case of its own, closed on every axis.  Periodic
    axes wrap; closed axes are cut at the domain edge, which then stays the real
    edge.  Returns (window case, per-axis global indices, per-axis position of
    the centre inside the window)."""
    shape, D = tuple(c["shape"]), len(c["shape"])
    idx, pos = [], []
    for d in range(D):
        n, lo, hi = shape[d], centre[d] - half, centre[d] + half + 1
        if c["periodic"][d]:
            ids = np.arange(lo, hi) % n
            pos.append(half)
        else:
            ids = np.arange(max(lo, 0), min(hi, n))
            pos.append(centre[d] - max(lo, 0))
        idx.append(ids)
    sel = np.ix_(*idx[::-1])                 # arrays are (z,) y, x
    w = dict(c, shape=tuple(len(i) for i in idx), periodic=(False,) * D,
             mask=np.ascontiguousarray(c["mask"][sel]),
             phi0=np.ascontiguousarray(c["phi0"][sel]))
    return w, idx, pos
